// Pieces shared by the chi0 tiles (internal): LDS DMA, waits, the per-chunk
// weights, the fold of the accumulators into FP64 partials and the
// XCD-aware workgroup order.  A tile configuration C
// provides kThreads (threads per workgroup), kWBlock (frequencies per
// workgroup), kChunk (transitions per chunk), kNW (weights per thread) and
// kWPart (fewer weights than threads).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

namespace tdx {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Chunks summed in FP32 between folds.  Every fold is a read-modify-write of
// the tile's FP64 partial, and the tiles running side by side fold at about
// the same time, so a fold costs a burst of HBM traffic; 1024 chunks keep
// that near 1 % of the kernel's time (it was 5 % at 256) while an FP32 run
// still adds at most 2^15 transitions.
constexpr int kFoldChunks = 1024;

// LDS index (float2 units) of the weight of transition tl of a chunk and
// frequency w of the workgroup: the four groups of four transitions that one
// 16-transition K-step reads side by side are adjacent.
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

// Wait until at most N of them are outstanding (they complete in issue
// order): vmcnt is split over bits 3:0 and 15:14 of the immediate.
template <int N>
__device__ inline void wait_vm_n() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
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
    const int tl = std::min(tw + (C::kThreads / C::kWBlock) * i, C::kChunk - 1);
    const long long t = std::min(tc + tl, t_max);
    pw.d[i] = delta[t];
    pw.f[i] = df[t];
  }
}

// ... and into LDS: w - delta in FP64 (it may cancel), the rest in FP32
// (relative error ~1e-7, far below the 2^-16 of the split products); zero
// past the end of the slice or of the frequency grid.  For a time-reversal
// paired list the weight is 2 df delta / D with
// D = (w + i eta)^2 - delta^2 = (w - delta)(w + delta) - eta^2 + 2 i w eta,
// whose real part is formed in FP64 for the same reason.
template <class C>
__device__ inline void store_weights(const Weights<C> &pw, float2 *wt, double om, bool w_ok,
                                     double eta, int paired, int tid, long long tc,
                                     long long t_hi) {
  const int tw = tid / C::kWBlock, wi = tid % C::kWBlock;
  const float etaf = (float)eta;
#pragma unroll
  for (int i = 0; i < C::kNW; ++i) {
    const int tl = tw + (C::kThreads / C::kWBlock) * i;
    if (C::kWPart && tl >= C::kChunk) break;
    const bool ok = tc + tl < t_hi && w_ok;
    float2 v;
    if (paired) {
      const float dr = (float)((om - pw.d[i]) * (om + pw.d[i]) - eta * eta);
      const float di = (float)(2.0 * om * eta);
      const float sc = (float)(2.0 * pw.f[i] * pw.d[i]) * __builtin_amdgcn_rcpf(fmaf(dr, dr, di * di));
      v = make_float2(sc * dr, -sc * di);
    } else {
      const float x = (float)(om - pw.d[i]);
      const float sc = (float)pw.f[i] * __builtin_amdgcn_rcpf(fmaf(x, x, etaf * etaf));
      v = make_float2(sc * x, -sc * etaf);
    }
    wt[wt_index<C>(tl, wi)] = ok ? v : make_float2(0.f, 0.f);
  }
}

// Fold the accumulators (FP32, or FP64 for the FP64 tile) into the tile's
// FP64 partial in global memory (the workgroup owns that region): the first
// fold stores, later ones add.  D[row][col] of a 16x16 MFMA: element j of
// lane l is column l%16 and row 4(l/16) + j (FP32 and bf16 forms) or
// l/16 + 4j (FP64 form, F64_ROWS).
template <int WPW, int SUB, class V = f32x4, bool F64_ROWS = false>
__device__ inline void fold(V (&ar)[WPW][SUB], V (&ai)[WPW][SUB], double2 *part, int n_w,
                            int n_g, int w0, int row0, int col0, int lane, int wave, bool first) {
#pragma unroll
  for (int i = 0; i < WPW; ++i) {
    const int w = w0 + wave * WPW + i;
#pragma unroll
    for (int b = 0; b < SUB; ++b) {
      const int col = col0 + b * 16 + (lane & 15);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = row0 + (F64_ROWS ? (lane >> 4) + 4 * j : 4 * (lane >> 4) + j);
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
      ar[i][b] = V{0, 0, 0, 0};
      ai[i][b] = V{0, 0, 0, 0};
    }
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

}  // namespace
}  // namespace tdx
