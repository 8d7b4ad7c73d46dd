// Split-BF16 chi0 contraction on the 16x16x32 bf16 MFMA of gfx950.
//
// Every real operand x is carried as x = hi + lo (bf16, round to nearest
// even) and a product as hi*hi' + hi*lo' + lo*hi' accumulated in FP32; the
// dropped lo*lo' term and the roundings leave a relative error near 2^-16
// per product.  The left operand A = w_t(w) rho_t(G) is formed in FP32 from
// the FP64 weight and the stored pair density, then split.
//
// One MFMA covers K = 32 reals = 16 transitions with (re, im) interleaved.
// With a = w_t rho_t(G) and b = rho_t(G'), chi0(G, G') sums a conj(b):
//   A[G][2t + p]     = (Re a, Im a),   A_rot[G][2t + p] = (Im a, -Re a),
//   B[2t + p][G']    = (Re b, Im b),
// so that A B accumulates Re chi0 and A_rot B accumulates Im chi0.  The
// rotation is applied to A, which is formed in registers anyway (A_rot is
// the split of (Im a, -Re a), exactly the rotated split of A because
// rounding to nearest even is odd-symmetric), so B carries two components
// (hi, lo) and no rotated copies.
//
// A tile is 16 G x (16 NSUB) G' for 4 WPW frequencies (4 waves x WPW) over
// one slice of transitions.  The pair densities arrive in a layout made for
// this kernel: per quad of transitions and column, the 16-byte groups hi and
// lo, so that one 16-byte-per-lane global-to-LDS transfer fills one
// lane-ordered B fragment, and the FP32 rho rows for the left operand.  Per
// chunk of CHUNK transitions the fragments and rho rows are copied into LDS
// with no register staging and no arithmetic; only the weights pass through
// registers.  The next chunk's transfers are in flight while the current
// chunk runs (two LDS buffers).  The number of 16-column blocks of a tile is
// a compile-time constant (the ragged last tile of a row runs its own
// instance), so the step body is one basic block.  Sums run in FP32 over 256
// chunks and are folded into the tile's FP64 partial; slices are reduced in
// FP64 in a fixed order, so results do not depend on which workgroup ran
// which tile.
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
  static constexpr int kSub = SUB;
  static constexpr int kCols = 16 * SUB;   // G' per tile
  static constexpr int kChunk = CHUNK;
  static constexpr int kSteps = CHUNK / 16;
  static constexpr int kBWords = kSteps * SUB * 2 * 64 * 4;  // [step][sub][comp][lane][4]
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

// cvt_pk(a, -b) with the negation as a source modifier of the conversion
// (the compiler would spend a separate sign flip on it)
__device__ inline unsigned int cvt_pk_neg_b(float a, float b) {
  unsigned int r;
  asm("v_cvt_pk_bf16_f32 %0, %1, -%2" : "=v"(r) : "v"(a), "v"(b));
  return r;
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

// LDS DMA of one chunk: the B fragments and the FP32 rho rows of CHUNK
// transitions.  The pair-density buffer carries a zero chunk past its last
// transition, so whole chunks are read without clamping.  The 1 KB transfers
// of a chunk are numbered B first, then rho, and dealt to the four waves in
// turn (transfer x = 4 slot + wave).
//  - B: block (s, b, comp) is the lane-ordered fragment of K-step s,
//    16-column block b and component comp (hi, lo).  Lane (kq = l/16,
//    c16 = l%16) copies the 16-byte word group of transitions
//    tc + 16 s + 4 kq .. +3 at column col0 + 16 b + c16.
//  - rho: block d holds float2 slots 64 d .. 64 d + 63 of the layout
//    rho_index; lane l copies rows row0 + 2 m, +1 (m = l & 7) of transition
//    tc + 16 (d/2) + 2 (d&1) + h + 4 kq2 (h = l/32, kq2 = l/8 & 3).
// Both kinds of source advance by 8 CHUNK ld bytes per chunk (CHUNK/4 quads
// of 2 x ld 16-byte groups, or CHUNK rows of ld 8-byte values), so each slot
// keeps the lane's address for the tile's first chunk and adds one uniform
// offset per chunk; the LDS destination of a slot is fixed.
template <class C, int NSUB>
struct DmaPlan {
  static constexpr int kB = C::kSteps * NSUB * 2, kT = kB + C::kChunk / 8;
  static constexpr int kSlots = (kT + 3) / 4;
  const unsigned char *src[kSlots];
  int dst[kSlots];  // word offset in a buffer
  bool last_ok;     // the last slot holds a transfer for this wave

  __device__ inline DmaPlan(const unsigned char *P2, const unsigned char *R, int ld,
                            long long t0, int col0, int row0, int wave, int lane) {
    const int kq = lane >> 4;
    const size_t lane_b = (size_t)(2 * kq * ld + (lane & 15)) * 16;
    const size_t lane_r = (size_t)(((lane >> 5) + 4 * ((lane >> 3) & 3)) * ld + 2 * (lane & 7)) * 8;
#pragma unroll
    for (int i = 0; i < kSlots; ++i) {
      const int x = 4 * i + wave;  // uniform across the wave
      if (x < kB) {
        const int m = x >> 1, comp = x & 1;
        const int st = m / NSUB, b = m % NSUB;
        src[i] = P2 + ((((size_t)(t0 >> 2) + 4 * st) * 2 + comp) * ld + col0 + 16 * b) * 16 +
                 lane_b;
        dst[i] = ((st * C::kSub + b) * 2 + comp) * 256;
      } else {
        const int d = std::min(x, kT - 1) - kB;
        src[i] = R + ((size_t)(t0 + 16 * (d >> 1) + 2 * (d & 1)) * ld + row0) * 8 + lane_r;
        dst[i] = C::kBWords + d * 256;
      }
    }
    last_ok = 4 * (kSlots - 1) + wave < kT;
  }

  // the chunk `off` bytes (8 CHUNK ld per chunk) past the first one
  __device__ inline void issue(size_t off, unsigned int *buf) const {
#pragma unroll
    for (int i = 0; i < kSlots; ++i)
      if (i < kSlots - 1 || (kT % 4 == 0) || last_ok) dma16(src[i] + off, buf + dst[i]);
  }
};

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

// One tile: rows row0..row0+15, columns col0..col0+16*NSUB-1, frequencies
// w0..w0+kWBlock-1, transitions [t_lo, t_hi).  Sums run in FP32 for at most
// kFoldChunks chunks and are folded into part (the slice's [n_w][n_g][n_g]
// block, FP64) between runs.
template <int WPW, int SUB, int CHUNK, int NSUB>
__device__ __attribute__((always_inline)) void chi0_tile(
    unsigned int *lds, const void *P, const void *R, int ld, const double *delta,
    const double *df, long long n_trans, long long t_lo, long long t_hi, const double *omega,
    int n_w, double eta, int n_g, int w0, int row0, int col0, double2 *part) {
  typedef Cfg<WPW, SUB, CHUNK> C;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int kq = lane >> 4;

  f32x4 ar[WPW][NSUB], ai[WPW][NSUB];
#pragma unroll
  for (int i = 0; i < WPW; ++i)
#pragma unroll
    for (int b = 0; b < NSUB; ++b) {
      ar[i][b] = f32x4{0, 0, 0, 0};
      ai[i][b] = f32x4{0, 0, 0, 0};
    }

  const long long t_max = n_trans - 1;
  const DmaPlan<C, NSUB> dma((const unsigned char *)P, (const unsigned char *)R, ld, t_lo, col0,
                             row0, wave, lane);
  const size_t chunk_bytes = (size_t)8 * CHUNK * ld;
  Weights<C> pw;
  const int wi = w0 + tid % C::kWBlock;
  const bool w_ok = wi < n_w;
  const double om = omega[std::min(wi, n_w - 1)];
  const float etaf = (float)eta;
  dma.issue(0, lds);
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
        dma.issue((size_t)((nx - t_lo) / CHUNK) * chunk_bytes, lds + (cur ^ 1) * C::kBufWords);
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
        // A and A_rot of the WPW frequencies, split: (hi, lo) words per
        // transition j of the lane's quad
        u32x4 ah[WPW], al[WPW], rh[WPW], rl[WPW];
#pragma unroll
        for (int i = 0; i < WPW; ++i) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float2 w = wt[((s * 4 + j) * C::kWBlock + wave * WPW + i) * 4 + kq];
            const float are = fmaf(w.x, rho[j].x, -w.y * rho[j].y);
            const float aim = fmaf(w.x, rho[j].y, w.y * rho[j].x);
            const unsigned int h = cvt_pk(are, aim);
            const float dre = are - lo_f(h), dim = aim - hi_f(h);
            ah[i][j] = h;
            al[i][j] = cvt_pk(dre, dim);
            rh[i][j] = cvt_pk_neg_b(aim, are);
            rl[i][j] = cvt_pk_neg_b(dim, dre);
          }
        }
#pragma unroll
        for (int b = 0; b < NSUB; ++b) {
          const u32x4 *bp = bfr + ((s * SUB + b) * 2) * 64 + lane;
          const bf16x8 bh = as_bf16x8(bp[0]), bl = as_bf16x8(bp[64]);
#pragma unroll
          for (int i = 0; i < WPW; ++i) {
            f32x4 cr = ar[i][b], ci = ai[i][b];
            cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah[i]), bh, cr, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(rh[i]), bh, ci, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah[i]), bl, cr, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(rh[i]), bl, ci, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(al[i]), bh, cr, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(rl[i]), bh, ci, 0, 0, 0);
            ar[i][b] = cr;
            ai[i][b] = ci;
          }
        }
      }
      if (more) store_weights<C>(pw, lds + (cur ^ 1) * C::kBufWords, om, w_ok, etaf, tid, nx, t_hi);
      wait_vm();
      __syncthreads();
      cur ^= 1;
    }
    fold<WPW, NSUB>(ar, ai, part, n_w, n_g, w0, row0, col0, lane, wave, first);
    first = false;
  }
}

// The tile routine for the tile's number of 16-column blocks inside the
// padded basis (ld is a multiple of 16): full tiles run NSUB = SUB, the last
// tile of a row may run fewer.
template <int WPW, int SUB, int CHUNK, int NSUB = SUB>
__device__ __attribute__((always_inline)) void chi0_tile_n(
    int nsub, unsigned int *lds, const void *P, const void *R, int ld, const double *delta,
    const double *df, long long n_trans, long long t_lo, long long t_hi, const double *omega,
    int n_w, double eta, int n_g, int w0, int row0, int col0, double2 *part) {
  if constexpr (NSUB > 1) {
    if (nsub < NSUB) {
      chi0_tile_n<WPW, SUB, CHUNK, NSUB - 1>(nsub, lds, P, R, ld, delta, df, n_trans, t_lo, t_hi,
                                              omega, n_w, eta, n_g, w0, row0, col0, part);
      return;
    }
  }
  chi0_tile<WPW, SUB, CHUNK, NSUB>(lds, P, R, ld, delta, df, n_trans, t_lo, t_hi, omega, n_w,
                                   eta, n_g, w0, row0, col0, part);
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
  const int col0 = gc * C::kCols;
  chi0_tile_n<WPW, SUB, CHUNK>(std::min(SUB, (ld - col0) / 16), lds, P, R, ld, delta, df, n_trans,
                               t_lo, t_hi, omega, n_w, eta, n_g, bx * C::kWBlock, gb * 16, col0,
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
    const int col0 = tl.gc * C::kCols;
    chi0_tile_n<WPW, SUB, CHUNK>(std::min(SUB, (it.ld - col0) / 16), lds, it.P, it.R, it.ld,
                                 it.delta, it.df, it.n_trans, t_lo, t_hi, it.omega, it.n_w,
                                 it.eta, it.n_g, tl.wblk * C::kWBlock, tl.gb * 16, col0,
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
                             TDX_V(2, 4, 32, 2), TDX_V(2, 9, 16, 2), TDX_V(2, 8, 32, 2)};
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
