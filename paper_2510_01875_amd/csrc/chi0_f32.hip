// FP32 chi0 contraction on the 16x16x4 FP32 MFMA of gfx950.
//
// The complex contraction is one real GEMM as in the split-BF16 tile: one
// K-step of 4 covers 2 transitions with (re, im) interleaved.  With
// a = w_t(w) rho_t(G) and b = rho_t(G'):
//   A[G][2t + p]   = (Re a, Im a),   A_rot[G][2t + p] = (Im a, -Re a),
//   B[2t + p][G']  = (Re b, Im b),
// A B accumulates Re chi0 and A_rot B accumulates Im chi0, in FP32; the
// accumulators are folded into the tile's FP64 partial every 128 chunks and
// slices are reduced in FP64 in a fixed order (bitwise reproducible).
//
// Lane l of an MFMA holds A[l%16][l/16] and B[l/16][l%16]: transition
// 2s + (l/16)/2, component (l/16)%2.  A is formed in registers from the FP32
// rho row and the FP32 weight (FP64 for w - delta), once per K-step and
// frequency, and reused over every column block of the tile; an MFMA of this
// shape runs long enough that the formation costs nothing.  The FP32 rows of
// the pair-density buffer ([T][ld] complex64, no padding) are copied into LDS
// by global-to-LDS transfers of 16 bytes per lane: per chunk the tile's 16
// rows (for A) and its 16 NSUB columns (for B) of CHUNK transitions; rows past
// the end of the list are clamped to the last one (their weights are zero).
#include <algorithm>
#include <cmath>

#include "chi0_tile.h"
#include "internal.h"

namespace tdx {
namespace {

template <int WPW, int SUB, int CHUNK>
struct CfgF32 {
  static constexpr int kWBlock = 4 * WPW;           // frequencies per workgroup
  static constexpr int kSub = SUB;
  static constexpr int kCols = 16 * SUB;            // G' per tile
  static constexpr int kChunk = CHUNK;
  static constexpr int kSteps = CHUNK / 2;          // K-steps of two transitions
  static constexpr int kBWords = CHUNK * kCols * 2;  // [t][16 NSUB] complex FP32
  static constexpr int kRhoWords = CHUNK * 16 * 2;   // [t][16] complex FP32
  static constexpr int kWtWords = CHUNK * kWBlock * 2;
  static constexpr int kBufWords = kBWords + kRhoWords + kWtWords;
  static constexpr bool kWPart = CHUNK * kWBlock < 256;
  static constexpr int kNW = kWPart ? 1 : CHUNK * kWBlock / 256;
  static_assert(256 % kWBlock == 0 && CHUNK % 16 == 0, "tile must divide the block");
};

constexpr int kF32FoldChunks = 128;  // chunks summed in FP32 between folds

// LDS transfers of one chunk: the B rows (CHUNK x 16 NSUB complex, row
// stride 16 NSUB) and the rho rows (CHUNK x 16), in 1 KB pieces dealt to the
// waves in turn.  Lane l of piece j copies LDS bytes 1024 j + 16 l; its
// source row and byte within the row are fixed per slot.
template <class C, int NSUB>
struct DmaPlanF32 {
  static constexpr int kRowB = 16 * NSUB * 8, kRowR = 16 * 8;  // bytes per row
  static constexpr int kB = C::kChunk * kRowB / 1024, kR = C::kChunk * kRowR / 1024;
  static constexpr int kT = kB + kR, kSlots = (kT + 3) / 4;
  int row[kSlots];       // row of the chunk the lane copies from
  unsigned col[kSlots];  // byte offset within that row (from col0 or row0)
  int dst[kSlots];       // word offset in a buffer
  bool is_r[kSlots], ok[kSlots];

  __device__ inline DmaPlanF32(int wave, int lane) {
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
          P + ((size_t)t * ld + (is_r[i] ? row0 : col0)) * 8 + col[i];
      dma16(src, buf + dst[i]);
    }
  }
};

// One tile: rows row0..row0+15, columns col0..col0+16 NSUB-1, frequencies
// w0..w0+kWBlock-1, transitions [t_lo, t_hi).
template <int WPW, int SUB, int CHUNK, int NSUB>
__device__ __attribute__((always_inline)) void chi0_tile_f32(
    unsigned int *lds, const void *P, int ld, const double *delta, const double *df, int paired,
    long long n_trans, long long t_lo, long long t_hi, const double *omega, int n_w, double eta,
    int n_g, int w0, int row0, int col0, double2 *part) {
  typedef CfgF32<WPW, SUB, CHUNK> C;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int tau = lane >> 5, comp = (lane >> 4) & 1, c16 = lane & 15;

  f32x4 ar[WPW][NSUB], ai[WPW][NSUB];
#pragma unroll
  for (int i = 0; i < WPW; ++i)
#pragma unroll
    for (int b = 0; b < NSUB; ++b) {
      ar[i][b] = f32x4{0, 0, 0, 0};
      ai[i][b] = f32x4{0, 0, 0, 0};
    }

  const unsigned char *Pb = (const unsigned char *)P;
  const long long t_max = n_trans - 1;
  const DmaPlanF32<C, NSUB> dma(wave, lane);
  Weights<C> pw;
  const int wi = w0 + tid % C::kWBlock;
  const bool w_ok = wi < n_w;
  const double om = omega[std::min(wi, n_w - 1)];
  dma.issue(Pb, ld, col0, row0, t_lo, t_max, lds);
  load_weights<C>(pw, delta, df, t_lo, t_max, tid);
  store_weights<C>(pw, (float2 *)(lds + C::kBWords + C::kRhoWords), om, w_ok, eta, paired, tid,
                   t_lo, t_hi);
  wait_vm();
  __syncthreads();
  int cur = 0;
  bool first = true;
  constexpr long long kRun = (long long)kF32FoldChunks * CHUNK;
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
      const float *bq = (const float *)buf;
      const float2 *rq = (const float2 *)(buf + C::kBWords);
      const float2 *wt = (const float2 *)(buf + C::kBWords + C::kRhoWords);
#pragma unroll 2
      for (int s = 0; s < C::kSteps; ++s) {
        const int tl = 2 * s + tau;
        const float2 rho = rq[tl * 16 + c16];
        float a[WPW], r[WPW];
#pragma unroll
        for (int i = 0; i < WPW; ++i) {
          const float2 w = wt[wt_index<C>(tl, wave * WPW + i)];
          const float are = fmaf(w.x, rho.x, -w.y * rho.y);
          const float aim = fmaf(w.x, rho.y, w.y * rho.x);
          a[i] = comp ? aim : are;
          r[i] = comp ? -are : aim;
        }
#pragma unroll
        for (int b = 0; b < NSUB; ++b) {
          const float bv = bq[(tl * 16 * NSUB + b * 16 + c16) * 2 + comp];
#pragma unroll
          for (int i = 0; i < WPW; ++i) {
            ar[i][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], bv, ar[i][b], 0, 0, 0);
            ai[i][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(r[i], bv, ai[i][b], 0, 0, 0);
          }
        }
      }
      if (more)
        store_weights<C>(pw, (float2 *)(lds + (cur ^ 1) * C::kBufWords + C::kBWords + C::kRhoWords),
                         om, w_ok, eta, paired, tid, nx, t_hi);
      wait_vm();
      __syncthreads();
      cur ^= 1;
    }
    fold<WPW, NSUB>(ar, ai, part, n_w, n_g, w0, row0, col0, lane, wave, first);
    first = false;
  }
}

template <int WPW, int SUB, int CHUNK, int NSUB = SUB>
__device__ __attribute__((always_inline)) void chi0_tile_f32_n(
    int nsub, unsigned int *lds, const void *P, int ld, const double *delta, const double *df,
    int paired, long long n_trans, long long t_lo, long long t_hi, const double *omega, int n_w,
    double eta, int n_g, int w0, int row0, int col0, double2 *part) {
  if constexpr (NSUB > 1) {
    if (nsub < NSUB) {
      chi0_tile_f32_n<WPW, SUB, CHUNK, NSUB - 1>(nsub, lds, P, ld, delta, df, paired, n_trans,
                                                  t_lo, t_hi, omega, n_w, eta, n_g, w0, row0,
                                                  col0, part);
      return;
    }
  }
  chi0_tile_f32<WPW, SUB, CHUNK, NSUB>(lds, P, ld, delta, df, paired, n_trans, t_lo, t_hi, omega,
                                       n_w, eta, n_g, w0, row0, col0, part);
}

// One tile per workgroup; logical tile = (frequency block fastest, then
// (G block, G' block), then slice), XCD-aware as in the split-BF16 grid.
template <int WPW, int SUB, int CHUNK>
__global__ void __launch_bounds__(256, 2)
    k_chi0_f32(const void *P, int ld, const double *delta, const double *df, int paired,
               long long n_trans, long long slice_len, const double *omega, int n_w, double eta,
               int n_g, int ncb, double2 *part) {
  typedef CfgF32<WPW, SUB, CHUNK> C;
  extern __shared__ unsigned int lds[];
  const int nx = gridDim.x, ny = gridDim.y;
  const int id = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
  const int L = xcd_logical(id, nx * ny * gridDim.z);
  const int bx = L % nx, by = (L / nx) % ny, bz = L / (nx * ny);
  const int gb = by / ncb, gc = by % ncb;
  const long long t_lo = (long long)bz * slice_len;
  const long long t_hi = std::min(n_trans, t_lo + slice_len);
  const int col0 = gc * C::kCols;
  chi0_tile_f32_n<WPW, SUB, CHUNK>(std::min(SUB, (ld - col0) / 16), lds, P, ld, delta, df, paired,
                                   n_trans, t_lo, t_hi, omega, n_w, eta, n_g, bx * C::kWBlock,
                                   gb * 16, col0, part + (size_t)bz * n_w * n_g * n_g);
}

constexpr int kF32Wpw = 4, kF32Sub = 3, kF32Chunk = 32;

}  // namespace

// Tile shape of the FP32 contraction: frequencies and G' columns per
// workgroup, transitions per chunk (slices are multiples of it).
void chi0_f32_shape(int *wblock, int *cols, int *chunk) {
  *wblock = 4 * kF32Wpw;
  *cols = 16 * kF32Sub;
  *chunk = kF32Chunk;
}

int chi0_f32_launch(const void *P, int ld, const double *delta, const double *df, int paired,
                    long long n_trans, long long slice_len, int slices, const double *omega,
                    int n_w, double eta, int n_g, double2 *part, hipStream_t s) {
  typedef CfgF32<kF32Wpw, kF32Sub, kF32Chunk> C;
  const void *fn = (const void *)k_chi0_f32<kF32Wpw, kF32Sub, kF32Chunk>;
  const size_t lds = (size_t)2 * C::kBufWords * 4;
  const int nblk = ld / 16, ncb = (ld + C::kCols - 1) / C::kCols;
  dim3 grid((n_w + C::kWBlock - 1) / C::kWBlock, nblk * ncb, (unsigned)slices);
  TDX_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL((k_chi0_f32<kF32Wpw, kF32Sub, kF32Chunk>), grid, dim3(256), lds, s, P, ld,
                     delta, df, paired, n_trans, slice_len, omega, n_w, eta, n_g, ncb, part);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

}  // namespace tdx
