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
// chunk runs (two or three LDS buffers); they are issued one per 16-column
// block of the current chunk, since a burst of them stalls the MFMAs of
// every wave on the CU.  The number of 16-column blocks of a tile is
// a compile-time constant (the ragged last tile of a row runs its own
// instance), so the step body is one basic block.  Sums run in FP32 over 1024
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
#include "chi0_tile.h"
#include "internal.h"

namespace tdx {
namespace {

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int WPW, int SUB, int CHUNK, int NW = 4>
struct Cfg {
  static constexpr int kWaves = NW;        // waves per workgroup
  static constexpr int kThreads = 64 * NW;
  static constexpr int kWBlock = NW * WPW;  // frequencies per tile
  static constexpr int kSub = SUB;
  static constexpr int kCols = 16 * SUB;   // G' per tile
  static constexpr int kChunk = CHUNK;
  static constexpr int kSteps = CHUNK / 16;
  static constexpr int kBWords = kSteps * SUB * 2 * 64 * 4;  // [step][sub][comp][lane][4]
  static constexpr int kRhoWords = CHUNK * 16 * 2;           // [t][row] float2
  static constexpr int kWtWords = CHUNK * kWBlock * 2;       // [t][w] float2
  static constexpr int kBufWords = kBWords + kRhoWords + kWtWords;
  // weights per thread; when the chunk holds fewer weights than threads only
  // the first CHUNK * kWBlock threads store one
  static constexpr bool kWPart = CHUNK * kWBlock < kThreads;
  static constexpr int kNW = kWPart ? 1 : CHUNK * kWBlock / kThreads;
  static_assert(kThreads % kWBlock == 0 && CHUNK % 16 == 0, "tile must divide the block");
};

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

// LDS index (float2 units) of rho(tl, row): the four transition groups kq
// that one MFMA K-step reads side by side are adjacent, so a read
// instruction touches consecutive words.
__device__ inline int rho_index(int tl, int row) {
  return (((tl >> 4) * 4 + (tl & 3)) * 4 + ((tl & 15) >> 2)) * 16 + row;
}
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
  static constexpr int kSlots = (kT + C::kWaves - 1) / C::kWaves;
  static constexpr int kIssued = kT / C::kWaves;  // transfers every wave issues per chunk
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
      const int x = C::kWaves * i + wave;  // uniform across the wave
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
    last_ok = C::kWaves * (kSlots - 1) + wave < kT;
  }

  // the chunk `off` bytes (8 CHUNK ld per chunk) past the first one
  __device__ inline void issue(size_t off, unsigned int *buf) const {
#pragma unroll
    for (int i = 0; i < kSlots; ++i) issue_slot(i, off, buf);
  }
  // one slot of it (i a compile-time constant after unrolling)
  __device__ inline void issue_slot(int i, size_t off, unsigned int *buf) const {
    if (i < kSlots && (i < kSlots - 1 || (kT % C::kWaves == 0) || last_ok))
      dma16(src[i] + off, buf + dst[i]);
  }
};

// Rows of a tail tile.  When n_g is not a multiple of 16 the basis rows (and
// columns) nm .. n_g - 1, nm = 16 floor(n_g / 16), would fill only part of a
// 16-row MFMA block (and a whole last block that would be a column tile of
// its own is taken the same way, nm = n_g - 16).  chi0 = H_R + i H_A with the Hermitian
//   H_R = pref sum_t Re(w_t) rho_t rho_t^H,  H_A = pref sum_t Im(w_t) rho_t rho_t^H,
// so the main tiles cover rows and columns [0, nm) only, and tail tiles
// compute the rows nm + g of H_R and H_A over every column: virtual rows
// r = (w tail + g) 2 + p (p = 0: weight Re w_t(w), p = 1: Im w_t(w)) packed
// 16 to an MFMA block across frequencies.  Those rows give chi0's rows
// nm + g directly and its columns nm + g through H = H^H (the reduction
// assembles them).
struct TailGeom {
  int nm, tail;     // first tail row of the basis and the tail row count
  int r0;           // first virtual row of the workgroup
  double2 *tpart;   // the slice's [n_w][tail][2][ld] FP64 partial
};

// Fold of a tail tile: output row 4(l/16) + j of block i is virtual row
// r0 + 16 (wave WPW + i) + 4 (l/16) + j.
template <int WPW, int SUB>
__device__ inline void fold_tail(f32x4 (&ar)[WPW][SUB], f32x4 (&ai)[WPW][SUB], const TailGeom &tg,
                                 int n_w, int ld, int col0, int lane, int wave, bool first) {
#pragma unroll
  for (int i = 0; i < WPW; ++i) {
#pragma unroll
    for (int b = 0; b < SUB; ++b) {
      const int col = col0 + b * 16 + (lane & 15);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int v = tg.r0 + 16 * (wave * WPW + i) + 4 * (lane >> 4) + j;
        const int w = v / (2 * tg.tail);
        if (w < n_w && col < ld) {
          double2 *d = tg.tpart + (size_t)v * ld + col;
          double2 x = make_double2((double)ar[i][b][j], (double)ai[i][b][j]);
          if (!first) {
            const double2 o = *d;
            x.x += o.x;
            x.y += o.y;
          }
          *d = x;
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
// block, FP64) between runs.  DEPTH LDS buffers: the transfers of chunk
// c + DEPTH - 1 are issued in iteration c; with three buffers the wait at the
// end of an iteration leaves that iteration's transfers in flight.  A tail
// tile (TAIL) runs the virtual rows of tg instead (row0 = tg.nm): each lane
// forms its own weights from the chunk's delta and df, which replace the
// weight table in LDS.
template <int WPW, int SUB, int CHUNK, int NSUB, int DEPTH, int NW, bool TAIL = false>
__device__ __attribute__((always_inline)) void chi0_tile(
    unsigned int *lds, const void *P, const void *R, int ld, const double *delta,
    const double *df, long long n_trans, long long t_lo, long long t_hi, const double *omega,
    int n_w, double eta, int paired, int n_g, int w0, int row0, int col0, double2 *part,
    TailGeom tg = TailGeom{}) {
  typedef Cfg<WPW, SUB, CHUNK, NW> C;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int kq = lane >> 4;
  static_assert(!TAIL || 2 * CHUNK * 8 <= C::kWtWords * 4, "delta/df of a chunk fit the weights");
  // tail tiles: the lane's virtual row of each of its WPW blocks
  double t_om[WPW];
  float t_di[WPW];
  int t_g[WPW];
  bool t_re[WPW], t_ok[WPW];
  if constexpr (TAIL) {
#pragma unroll
    for (int i = 0; i < WPW; ++i) {
      const int v = tg.r0 + 16 * (wave * WPW + i) + (lane & 15);
      const int w = v / (2 * tg.tail), rem = v % (2 * tg.tail);
      t_ok[i] = w < n_w;
      t_om[i] = omega[std::min(w, n_w - 1)];
      t_di[i] = (float)(2.0 * t_om[i] * eta);
      t_g[i] = rem >> 1;
      t_re[i] = (rem & 1) == 0;
    }
  }
  // tail tiles: delta and df of one chunk into LDS (thread tid < CHUNK takes
  // transition tid; zero past the slice, which zeroes the weight)
  double t_d = 0.0, t_f = 0.0;
  auto tail_load = [&](long long tc) {
    const long long t = tc + tid;
    const bool ok = tid < CHUNK && t < t_hi;
    t_d = ok ? delta[t] : 0.0;
    t_f = ok ? df[t] : 0.0;
  };
  auto tail_store = [&](unsigned int *buf) {
    double *dd = (double *)(buf + C::kBWords + C::kRhoWords);
    if (tid < CHUNK) {
      dd[tid] = t_d;
      dd[CHUNK + tid] = t_f;
    }
  };

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
#pragma unroll
  for (int k = 0; k < DEPTH - 1; ++k) {
    if (t_lo + k * CHUNK >= t_hi) break;
    dma.issue((size_t)k * chunk_bytes, lds + k * C::kBufWords);
    if constexpr (TAIL) {
      tail_load(t_lo + k * CHUNK);
      tail_store(lds + k * C::kBufWords);
    } else {
      load_weights<C>(pw, delta, df, t_lo + k * CHUNK, t_max, tid);
      store_weights<C>(pw, (float2 *)(lds + k * C::kBufWords + C::kBWords + C::kRhoWords), om,
                       w_ok, eta, paired, tid, t_lo + k * CHUNK, t_hi);
    }
  }
  wait_vm();
  __syncthreads();
  int cur = 0, ahead = DEPTH - 1;  // buffers of chunk c and of chunk c + DEPTH - 1
  bool first = true;
  constexpr long long kRun = (long long)kFoldChunks * CHUNK;
  for (long long rs = t_lo; rs < t_hi; rs += kRun) {
    const long long re = std::min(t_hi, rs + kRun);
    for (long long tc = rs; tc < re; tc += CHUNK) {
      const long long nx = tc + (DEPTH - 1) * CHUNK;
      const bool more = nx < t_hi;
      // weights first: a partial wait below leaves the transfers in flight
      if (more) {
        if constexpr (TAIL)
          tail_load(nx);
        else
          load_weights<C>(pw, delta, df, nx, t_max, tid);
      }
      // the transfers of chunk nx go out one slot per column block of the
      // first K-steps rather than all at once: a burst of them at the top of
      // the chunk stalls the MFMAs of every wave of the CU
      const size_t nx_off = (size_t)((nx - t_lo) / CHUNK) * chunk_bytes;
      unsigned int *nx_buf = lds + ahead * C::kBufWords;
      static_assert(DmaPlan<C, NSUB>::kSlots <= C::kSteps * NSUB, "a slot per column block");
      const unsigned int *buf = lds + cur * C::kBufWords;
      const u32x4 *bfr = (const u32x4 *)buf;
      const float2 *rq = (const float2 *)(buf + C::kBWords);
      const float2 *wt = (const float2 *)(buf + C::kBWords + C::kRhoWords);
#pragma unroll
      for (int s = 0; s < C::kSteps; ++s) {
        float2 rho[4];
        if constexpr (!TAIL) {
#pragma unroll
          for (int j = 0; j < 4; ++j) rho[j] = rq[(s * 4 + j) * 64 + lane];
        }
        // A and A_rot of the WPW frequencies, split: (hi, lo) words per
        // transition j of the lane's quad
        u32x4 ah[WPW], al[WPW], rh[WPW], rl[WPW];
#pragma unroll
        for (int i = 0; i < WPW; ++i) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            float are, aim;
            if constexpr (TAIL) {
              // the lane's weight, formed as store_weights forms it, then
              // its real (H_R) or imaginary (H_A) part times rho(nm + g)
              const double *dd = (const double *)wt;
              const int tl = 16 * s + 4 * kq + j;
              const double dl = dd[tl], fv = dd[CHUNK + tl];
              float wr, wim;
              if (paired) {
                const float dr = (float)((t_om[i] - dl) * (t_om[i] + dl) - eta * eta);
                const float sc = (float)(2.0 * fv * dl) *
                                 __builtin_amdgcn_rcpf(fmaf(dr, dr, t_di[i] * t_di[i]));
                wr = sc * dr;
                wim = -sc * t_di[i];
              } else {
                const float x = (float)(t_om[i] - dl), etaf = (float)eta;
                const float sc = (float)fv * __builtin_amdgcn_rcpf(fmaf(x, x, etaf * etaf));
                wr = sc * x;
                wim = -sc * etaf;
              }
              const float cw = t_ok[i] ? (t_re[i] ? wr : wim) : 0.f;
              const float2 rv = rq[(s * 4 + j) * 64 + kq * 16 + t_g[i]];
              are = cw * rv.x;
              aim = cw * rv.y;
            } else {
              const float2 w = wt[((s * 4 + j) * C::kWBlock + wave * WPW + i) * 4 + kq];
              are = fmaf(w.x, rho[j].x, -w.y * rho[j].y);
              aim = fmaf(w.x, rho[j].y, w.y * rho[j].x);
            }
            const unsigned int h = cvt_pk(are, aim);
            const float dre = are - lo_f(h), dim = aim - hi_f(h);
            ah[i][j] = h;
            al[i][j] = cvt_pk(dre, dim);
            rh[i][j] = cvt_pk_neg_b(aim, are);
            rl[i][j] = cvt_pk_neg_b(dim, dre);
          }
        }
        // B fragments one column block ahead: the reads of block b + 1 are
        // in flight while the MFMAs of block b run (a fence per block keeps
        // that order)
        bf16x8 bh[2], bl[2];
        {
          const u32x4 *bp = bfr + ((s * SUB) * 2) * 64 + lane;
          bh[0] = as_bf16x8(bp[0]);
          bl[0] = as_bf16x8(bp[64]);
        }
#pragma unroll
        for (int b = 0; b < NSUB; ++b) {
          if (b + 1 < NSUB) {
            const u32x4 *bp = bfr + ((s * SUB + b + 1) * 2) * 64 + lane;
            bh[(b + 1) & 1] = as_bf16x8(bp[0]);
            bl[(b + 1) & 1] = as_bf16x8(bp[64]);
          }
          if (more) dma.issue_slot(s * NSUB + b, nx_off, nx_buf);
#pragma unroll
          for (int i = 0; i < WPW; ++i) {
            f32x4 cr = ar[i][b], ci = ai[i][b];
            cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah[i]), bh[b & 1], cr, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(rh[i]), bh[b & 1], ci, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ah[i]), bl[b & 1], cr, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(rh[i]), bl[b & 1], ci, 0, 0, 0);
            cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(al[i]), bh[b & 1], cr, 0, 0, 0);
            ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(rl[i]), bh[b & 1], ci, 0, 0, 0);
            ar[i][b] = cr;
            ai[i][b] = ci;
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      if (more) {
        if constexpr (TAIL)
          tail_store(lds + ahead * C::kBufWords);
        else
          store_weights<C>(pw, (float2 *)(lds + ahead * C::kBufWords + C::kBWords + C::kRhoWords),
                           om, w_ok, eta, paired, tid, nx, t_hi);
      }
      if (DEPTH > 2 && more)
        wait_vm_n<DmaPlan<C, NSUB>::kIssued>();
      else
        wait_vm();
      __syncthreads();
      cur = cur == DEPTH - 1 ? 0 : cur + 1;
      ahead = ahead == DEPTH - 1 ? 0 : ahead + 1;
    }
    if constexpr (TAIL)
      fold_tail<WPW, NSUB>(ar, ai, tg, n_w, ld, col0, lane, wave, first);
    else
      fold<WPW, NSUB>(ar, ai, part, n_w, n_g, w0, row0, col0, lane, wave, first);
    first = false;
  }
}

// The tile routine for the tile's number of 16-column blocks inside the
// padded basis (ld is a multiple of 16): full tiles run NSUB = SUB, the last
// tile of a row may run fewer.
template <int WPW, int SUB, int CHUNK, int DEPTH, int NW, bool TAIL = false, int NSUB = SUB>
__device__ __attribute__((always_inline)) void chi0_tile_n(
    int nsub, unsigned int *lds, const void *P, const void *R, int ld, const double *delta,
    const double *df, long long n_trans, long long t_lo, long long t_hi, const double *omega,
    int n_w, double eta, int paired, int n_g, int w0, int row0, int col0, double2 *part,
    TailGeom tg = TailGeom{}) {
  if constexpr (NSUB > 1) {
    if (nsub < NSUB) {
      chi0_tile_n<WPW, SUB, CHUNK, DEPTH, NW, TAIL, NSUB - 1>(
          nsub, lds, P, R, ld, delta, df, n_trans, t_lo, t_hi, omega, n_w, eta, paired, n_g, w0,
          row0, col0, part, tg);
      return;
    }
  }
  chi0_tile<WPW, SUB, CHUNK, NSUB, DEPTH, NW, TAIL>(lds, P, R, ld, delta, df, n_trans, t_lo, t_hi,
                                                    omega, n_w, eta, paired, n_g, w0, row0, col0,
                                                    part, tg);
}

// ---------------------------------------------------------------------------
// Software-pipelined tile (one wave per SIMD).  While the MFMAs of K-step g
// run, the same wave forms the split left operand of step g + 1 in the VALU,
// so the two pipes overlap inside one wave.  With no second wave on the SIMD
// to cover a late transfer, the transfers run further ahead: B fragments in
// three buffers filled two chunks ahead, rho rows and weights (needed one
// chunk before their B, for the formation) in four slots filled three chunks
// ahead.  In iteration c:
//   load the weights of c+3; issue B(c+2) -> buffer (c+2)%3 and rho(c+3) ->
//   slot (c+3)%4; per K-step: MFMAs on A(g) and B(c) || form A(g+1) from
//   slot c%4 (slot (c+1)%4 for the last step); store the weights of c+3;
//   wait for this wave's transfers of iteration c-1 and older; barrier.
// Every buffer or slot written in iteration c was last read in iteration
// c-1, before the barrier that ends it, and every transfer read in iteration
// c was issued in iteration c-2 or earlier and waited for at the end of c-1.
// Two register sets hold A(g) and A(g+1), which needs the 512 registers of a
// lone wave.

// The split left operand of one K-step for the WPW frequencies of the wave:
// A[i][0..3] = hi, lo of (Re a, Im a) and of (Im a, -Re a).
template <class C, int WPW>
__device__ inline void form_a(u32x4 (&A)[WPW][4], const float2 *rq, const float2 *wt, int s,
                              int lane, int kq, int wave) {
  float2 rho[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) rho[j] = rq[(s * 4 + j) * 64 + lane];
#pragma unroll
  for (int i = 0; i < WPW; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float2 w = wt[((s * 4 + j) * C::kWBlock + wave * WPW + i) * 4 + kq];
      const float are = fmaf(w.x, rho[j].x, -w.y * rho[j].y);
      const float aim = fmaf(w.x, rho[j].y, w.y * rho[j].x);
      const unsigned int h = cvt_pk(are, aim);
      const float dre = are - lo_f(h), dim = aim - hi_f(h);
      A[i][0][j] = h;
      A[i][1][j] = cvt_pk(dre, dim);
      A[i][2][j] = cvt_pk_neg_b(aim, are);
      A[i][3][j] = cvt_pk_neg_b(dim, dre);
    }
  }
}

// One K-step of the pipelined tile: the MFMAs of step s on A (B from bfr)
// and, interleaved with them, the formation of An for step sn from rqn,
// wtn.  Per 16-column block: the B reads of the next block, the block's
// MFMAs, one element (i, j) of the formation; a scheduling fence after each
// block keeps the pieces in this order, so the VALU work of the formation
// issues between the MFMAs of the same wave.
template <class C, int WPW, int NSUB>
__device__ inline void step_pipe(f32x4 (&ar)[WPW][NSUB], f32x4 (&ai)[WPW][NSUB],
                                 const u32x4 (&A)[WPW][4], u32x4 (&An)[WPW][4],
                                 const u32x4 *bfr, int s, const float2 *rqn, const float2 *wtn,
                                 int sn, int lane, int kq, int wave) {
  float2 rho[4], w[WPW][4];
#pragma unroll
  for (int j = 0; j < 4; ++j) rho[j] = rqn[(sn * 4 + j) * 64 + lane];
#pragma unroll
  for (int i = 0; i < WPW; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) w[i][j] = wtn[((sn * 4 + j) * C::kWBlock + wave * WPW + i) * 4 + kq];
  auto element = [&](int e) {
    const int i = e / 4, j = e % 4;
    const float are = fmaf(w[i][j].x, rho[j].x, -w[i][j].y * rho[j].y);
    const float aim = fmaf(w[i][j].x, rho[j].y, w[i][j].y * rho[j].x);
    const unsigned int h = cvt_pk(are, aim);
    const float dre = are - lo_f(h), dim = aim - hi_f(h);
    An[i][0][j] = h;
    An[i][1][j] = cvt_pk(dre, dim);
    An[i][2][j] = cvt_pk_neg_b(aim, are);
    An[i][3][j] = cvt_pk_neg_b(dim, dre);
  };
  bf16x8 bh[2], bl[2];
  {
    const u32x4 *bp = bfr + ((s * C::kSub) * 2) * 64 + lane;
    bh[0] = as_bf16x8(bp[0]);
    bl[0] = as_bf16x8(bp[64]);
  }
#pragma unroll
  for (int b = 0; b < NSUB; ++b) {
    if (b + 1 < NSUB) {
      const u32x4 *bp = bfr + ((s * C::kSub + b + 1) * 2) * 64 + lane;
      bh[(b + 1) & 1] = as_bf16x8(bp[0]);
      bl[(b + 1) & 1] = as_bf16x8(bp[64]);
    }
#pragma unroll
    for (int i = 0; i < WPW; ++i) {
      f32x4 cr = ar[i][b], ci = ai[i][b];
      cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(A[i][0]), bh[b & 1], cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(A[i][2]), bh[b & 1], ci, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(A[i][0]), bl[b & 1], cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(A[i][2]), bl[b & 1], ci, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(A[i][1]), bh[b & 1], cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(A[i][3]), bh[b & 1], ci, 0, 0, 0);
      ar[i][b] = cr;
      ai[i][b] = ci;
    }
    if (b < 4 * WPW) element(b);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int e = NSUB; e < 4 * WPW; ++e) element(e);
}

// LDS DMA of the pipelined tile.  Transfers are dealt to the NW waves per
// kind: B transfer x = NW slot + wave (slots 0 .. kSB-1), rho transfer
// d = NW slot' + wave (the kSR slots after them), so every slot's kind is
// fixed at compile time; a slot is empty for a wave only when its kind's
// count is not a multiple of NW.
template <class C, int NSUB>
struct DmaPlanPipe {
  static constexpr int kW = C::kWaves;
  static constexpr int kB = C::kSteps * NSUB * 2, kR = C::kChunk / 8;
  static constexpr int kSB = (kB + kW - 1) / kW, kSR = (kR + kW - 1) / kW;
  // B and rho transfers that every wave issues per chunk (a lower bound for
  // the waves that also fill a last, partial slot)
  static constexpr int kIssuedB = kB / kW, kIssuedR = kR / kW;
  const unsigned char *base_b, *base_r;  // the tile's first chunk (uniform)
  unsigned off[kSB + kSR];               // the lane's byte offset per slot
  int dst[kSB + kSR];                    // word offset in a B buffer or a rho slot
  bool lastb_ok, lastr_ok;

  __device__ inline DmaPlanPipe(const unsigned char *P2, const unsigned char *R, int ld,
                                long long t0, int col0, int row0, int wave, int lane) {
    const int kq = lane >> 4;
    base_b = P2 + ((size_t)(t0 >> 2) * 2 * ld + col0) * 16;
    base_r = R + ((size_t)t0 * ld + row0) * 8;
    const unsigned lane_b = (unsigned)(2 * kq * ld + (lane & 15)) * 16u;
    const unsigned lane_r = (unsigned)(((lane >> 5) + 4 * ((lane >> 3) & 3)) * ld + 2 * (lane & 7)) * 8u;
#pragma unroll
    for (int i = 0; i < kSB; ++i) {
      const int x = std::min(kW * i + wave, kB - 1);
      const int m = x >> 1, comp = x & 1;
      const int st = m / NSUB, b = m % NSUB;
      off[i] = (unsigned)(((4 * st) * 2 + comp) * ld + 16 * b) * 16u + lane_b;
      dst[i] = ((st * C::kSub + b) * 2 + comp) * 256;
    }
#pragma unroll
    for (int i = 0; i < kSR; ++i) {
      const int d = std::min(kW * i + wave, kR - 1);
      off[kSB + i] = (unsigned)((16 * (d >> 1) + 2 * (d & 1)) * ld) * 8u + lane_r;
      dst[kSB + i] = d * 256;
    }
    lastb_ok = kW * (kSB - 1) + wave < kB;
    lastr_ok = kW * (kSR - 1) + wave < kR;
  }

  // B / rho of the chunk `pos` bytes past the tile's first one into buf
  __device__ inline void issue_b(size_t pos, unsigned int *buf) const {
    const unsigned char *b = base_b + pos;
#pragma unroll
    for (int i = 0; i < kSB; ++i)
      if (i < kSB - 1 || kB % kW == 0 || lastb_ok) dma16(b + off[i], buf + dst[i]);
  }
  __device__ inline void issue_r(size_t pos, unsigned int *buf) const {
    const unsigned char *r = base_r + pos;
#pragma unroll
    for (int i = 0; i < kSR; ++i)
      if (i < kSR - 1 || kR % kW == 0 || lastr_ok) dma16(r + off[kSB + i], buf + dst[kSB + i]);
  }
};

template <int WPW, int SUB, int CHUNK, int NW>
struct PipeLds {
  typedef Cfg<WPW, SUB, CHUNK, NW> C;
  static constexpr int kRW = C::kRhoWords + C::kWtWords;  // one rho/weight slot
  static constexpr int kBBufs = 3, kRWSlots = 4;
  static constexpr size_t kBytes = (size_t)(kBBufs * C::kBWords + kRWSlots * kRW) * 4;
};

template <int WPW, int SUB, int CHUNK, int NSUB, int NW>
__device__ __attribute__((always_inline)) void chi0_tile_pipe(
    unsigned int *lds, const void *P, const void *R, int ld, const double *delta,
    const double *df, long long n_trans, long long t_lo, long long t_hi, const double *omega,
    int n_w, double eta, int paired, int n_g, int w0, int row0, int col0, double2 *part) {
  typedef Cfg<WPW, SUB, CHUNK, NW> C;
  typedef PipeLds<WPW, SUB, CHUNK, NW> L;
  static_assert(C::kSteps % 2 == 0, "the A register sets alternate per K-step");
  unsigned int *bring = lds, *rwring = lds + L::kBBufs * C::kBWords;
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

  typedef DmaPlanPipe<C, NSUB> D;
  const long long t_max = n_trans - 1;
  const D dma((const unsigned char *)P, (const unsigned char *)R, ld, t_lo, col0, row0, wave,
              lane);
  const size_t chunk_bytes = (size_t)8 * CHUNK * ld;
  const long long n_chunks = (t_hi - t_lo + CHUNK - 1) / CHUNK;
  Weights<C> pw;
  const int wi = w0 + tid % C::kWBlock;
  const bool w_ok = wi < n_w;
  const double om = omega[std::min(wi, n_w - 1)];
  // buffers and slots by index (chunk k uses B buffer k % 3, slot k % 4)
  auto bbuf = [&](int i) { return bring + i * C::kBWords; };
  auto rbuf = [&](int i) { return rwring + i * L::kRW; };
  auto rho_of = [&](int i) { return (const float2 *)(rwring + i * L::kRW); };
  auto wt_of = [&](int i) { return (float2 *)(rwring + i * L::kRW + C::kRhoWords); };

  // prologue: B of chunks 0, 1; rho and weights of chunks 0, 1, 2
  for (int k = 0; k < 3 && k < n_chunks; ++k) {
    if (k < 2) dma.issue_b((size_t)k * chunk_bytes, bbuf(k));
    dma.issue_r((size_t)k * chunk_bytes, rbuf(k));
    load_weights<C>(pw, delta, df, t_lo + k * CHUNK, t_max, tid);
    store_weights<C>(pw, wt_of(k), om, w_ok, eta, paired, tid, t_lo + k * CHUNK, t_hi);
  }
  wait_vm();
  __syncthreads();
  u32x4 A0[WPW][4], A1[WPW][4];
  form_a<C, WPW>(A0, rho_of(0), wt_of(0), 0, lane, kq, wave);

  bool first = true;
  long long c = 0;
  int b0 = 0, b2 = 2;          // B buffers of chunks c, c+2
  int r0 = 0, r1 = 1, r3 = 3;  // rho/weight slots of chunks c, c+1, c+3
  for (long long run = 0; run < n_chunks; run += kFoldChunks) {
    const long long run_end = std::min(n_chunks, run + kFoldChunks);
    for (; c < run_end; ++c) {
      const bool more2 = c + 2 < n_chunks, more3 = c + 3 < n_chunks;
      // weights first: the wait at the end of the iteration may leave the
      // transfers issued after them in flight
      if (more3) load_weights<C>(pw, delta, df, t_lo + (c + 3) * CHUNK, t_max, tid);
      if (more2) dma.issue_b((size_t)(c + 2) * chunk_bytes, bbuf(b2));
      if (more3) dma.issue_r((size_t)(c + 3) * chunk_bytes, rbuf(r3));
      const u32x4 *bfr = (const u32x4 *)bbuf(b0);
#pragma unroll
      for (int s = 0; s < C::kSteps; s += 2) {
        // step s on A0 forming A1 (step s + 1 of this chunk); step s + 1 on
        // A1 forming A0 (the next step: of this chunk, or step 0 of the next)
        step_pipe<C, WPW, NSUB>(ar, ai, A0, A1, bfr, s, rho_of(r0), wt_of(r0), s + 1, lane, kq,
                                wave);
        if (s + 2 < C::kSteps)
          step_pipe<C, WPW, NSUB>(ar, ai, A1, A0, bfr, s + 1, rho_of(r0), wt_of(r0), s + 2, lane,
                                  kq, wave);
        else
          step_pipe<C, WPW, NSUB>(ar, ai, A1, A0, bfr, s + 1, rho_of(r1), wt_of(r1), 0, lane, kq,
                                  wave);
      }
      if (more3)
        store_weights<C>(pw, wt_of(r3), om, w_ok, eta, paired, tid, t_lo + (c + 3) * CHUNK, t_hi);
      // this iteration's transfers may stay in flight; older ones are done
      if (more2 && more3)
        wait_vm_n<D::kIssuedB + D::kIssuedR>();
      else
        wait_vm();
      __syncthreads();
      b0 = b0 == 2 ? 0 : b0 + 1;
      b2 = b2 == 2 ? 0 : b2 + 1;
      r0 = r1;
      r1 = (r1 + 1) & 3;
      r3 = (r3 + 1) & 3;
    }
    fold<WPW, NSUB>(ar, ai, part, n_w, n_g, w0, row0, col0, lane, wave, first);
    first = false;
  }
}

template <int WPW, int SUB, int CHUNK, int NW, int NSUB = SUB>
__device__ __attribute__((always_inline)) void chi0_tile_pipe_n(
    int nsub, unsigned int *lds, const void *P, const void *R, int ld, const double *delta,
    const double *df, long long n_trans, long long t_lo, long long t_hi, const double *omega,
    int n_w, double eta, int paired, int n_g, int w0, int row0, int col0, double2 *part) {
  if constexpr (NSUB > 1) {
    if (nsub < NSUB) {
      chi0_tile_pipe_n<WPW, SUB, CHUNK, NW, NSUB - 1>(nsub, lds, P, R, ld, delta, df, n_trans, t_lo,
                                                   t_hi, omega, n_w, eta, paired, n_g, w0, row0, col0,
                                                   part);
      return;
    }
  }
  chi0_tile_pipe<WPW, SUB, CHUNK, NSUB, NW>(lds, P, R, ld, delta, df, n_trans, t_lo, t_hi, omega,
                                        n_w, eta, paired, n_g, w0, row0, col0, part);
}

// The tile routine of a variant: plain (PIPE false, DEPTH buffers) or
// software-pipelined.
template <int WPW, int SUB, int CHUNK, bool PIPE, int DEPTH, int NW>
__device__ __attribute__((always_inline)) void run_tile(
    int nsub, unsigned int *lds, const void *P, const void *R, int ld, const double *delta,
    const double *df, long long n_trans, long long t_lo, long long t_hi, const double *omega,
    int n_w, double eta, int paired, int n_g, int w0, int row0, int col0, double2 *part) {
  if constexpr (PIPE)
    chi0_tile_pipe_n<WPW, SUB, CHUNK, NW>(nsub, lds, P, R, ld, delta, df, n_trans, t_lo, t_hi, omega,
                                      n_w, eta, paired, n_g, w0, row0, col0, part);
  else
    chi0_tile_n<WPW, SUB, CHUNK, DEPTH, NW>(nsub, lds, P, R, ld, delta, df, n_trans, t_lo, t_hi,
                                        omega, n_w, eta, paired, n_g, w0, row0, col0, part);
}

// The tail tile of a variant (plain tiles only: a pipelined variant keeps
// the padded rows and columns and has no tail tiles).
template <int WPW, int SUB, int CHUNK, bool PIPE, int DEPTH, int NW>
__device__ __attribute__((always_inline)) void run_tail_tile(
    int nsub, unsigned int *lds, const void *P, const void *R, int ld, const double *delta,
    const double *df, long long n_trans, long long t_lo, long long t_hi, const double *omega,
    int n_w, double eta, int paired, int n_g, int col0, const TailGeom &tg) {
  if constexpr (!PIPE)
    chi0_tile_n<WPW, SUB, CHUNK, DEPTH, NW, true>(nsub, lds, P, R, ld, delta, df, n_trans, t_lo,
                                                  t_hi, omega, n_w, eta, paired, n_g, 0, tg.nm,
                                                  col0, nullptr, tg);
}

// One tile per workgroup: the tail tiles first (logical tiles 0 .. n_tail - 1:
// virtual-row group fastest, then column tile, then slice; they hold the
// most column blocks), then the main tiles (frequency block fastest, then
// (G block, G' block), then slice), so one launch fills the chip with both.
// OCC = workgroups per CU: 2 for the
// plain tile (one wave per SIMD without pipelining leaves LDS and dependency
// latency exposed: about 60 % of the two-wave rate for 16 x 128 and 16 x 144
// tiles), 1 for the pipelined tile, whose two operand register sets need the
// 512 registers of a lone wave.
template <int WPW, int SUB, int CHUNK, int OCC, bool PIPE, int DEPTH, int NW>
__global__ void __launch_bounds__(64 * NW, OCC)
    k_chi0_bf16x3(const void *P, const void *R, int ld, const double *delta, const double *df,
                  long long n_trans, long long slice_len, const double *omega, int n_w,
                  double eta, int paired, int n_g, int lc, int nx, int ncb, int ny, int n_tail,
                  int ntg, int nct, int nm, int tail, double2 *part, double2 *tpart) {
  // main tiles: rows and columns [0, lc) (lc = ld, or nm when tail tiles
  // cover the rest); grid: n_tail + nx ny slices workgroups
  typedef Cfg<WPW, SUB, CHUNK, NW> C;
  extern __shared__ unsigned int lds[];
  // XCD x runs a contiguous range of logical tiles.  The tail tiles come
  // first in the logical order, so XCD 0's range holds them all; where they
  // would load it with more than a tenth of a range's work beyond the
  // others' (a tail tile costs about 1.35 main ones), each range starts with
  // an eighth of them instead (fcc_c2 q0, 240 tail tiles in ranges of 414:
  // 4 % faster; with 108 in ranges of 877 the spread took 40 % more L2
  // misses and 1 % longer, so smaller shares stay in XCD 0)
  const int id = blockIdx.x, per = gridDim.x / 8;
  const bool spread = (n_tail + 7) / 8 <= per && 7LL * n_tail > 2LL * per;
  int L;
  if (spread && id < 8 * per) {
    const int x = id % 8, j = id / 8;
    const int t0 = (int)((long long)n_tail * x / 8), t1 = (int)((long long)n_tail * (x + 1) / 8);
    L = j < t1 - t0 ? t0 + j : n_tail + x * per - t0 + (j - (t1 - t0));
  } else if (spread) {
    L = id;
  } else {
    L = xcd_logical(id, gridDim.x);
  }
  if (L < n_tail) {
    const int a = L % ntg, c = (L / ntg) % nct, bz = L / (ntg * nct);
    const long long t_lo = (long long)bz * slice_len;
    const long long t_hi = std::min(n_trans, t_lo + slice_len);
    const int col0 = c * C::kCols;
    const TailGeom tg{nm, tail, a * 16 * WPW * NW, tpart + (size_t)bz * n_w * tail * 2 * ld};
    run_tail_tile<WPW, SUB, CHUNK, PIPE, DEPTH, NW>(std::min(SUB, (ld - col0) / 16), lds, P, R,
                                                    ld, delta, df, n_trans, t_lo, t_hi, omega,
                                                    n_w, eta, paired, n_g, col0, tg);
    return;
  }
  const int Lm = L - n_tail;
  const int bx = Lm % nx, by = (Lm / nx) % ny, bz = Lm / (nx * ny);
  const int gb = by / ncb, gc = by % ncb;
  const long long t_lo = (long long)bz * slice_len;
  const long long t_hi = std::min(n_trans, t_lo + slice_len);
  const int col0 = gc * C::kCols;
  run_tile<WPW, SUB, CHUNK, PIPE, DEPTH, NW>(std::min(SUB, (lc - col0) / 16), lds, P, R, ld, delta, df,
                                  n_trans, t_lo, t_hi, omega, n_w, eta, paired, n_g, bx * C::kWBlock,
                                  gb * 16, col0, part + (size_t)bz * n_w * n_g * n_g);
}

template <int W, int S, int K, bool PIPE, int DEPTH, int NW>
constexpr size_t variant_lds() {
  if constexpr (PIPE)
    return PipeLds<W, S, K, NW>::kBytes;
  else
    return (size_t)DEPTH * Cfg<W, S, K, NW>::kBufWords * 4;
}

// Persistent form: a fixed grid (OCC workgroups per CU) takes tiles from
// the costliest-first tile list one at a time through an atomic counter, so
// a workgroup that finishes early takes the next tile.  Tiles in flight at
// one time are neighbours in the list, mostly of one slice, so they share
// its pair-density rows in L2 whichever XCD runs them.  Every workgroup
// leaves once the counter has passed the end; the last one out (counted in
// the second word) sets both words back to zero for the next launch, so the
// queue needs no clearing between launches or graph replays.  The tile
// index is passed on through one word after the tile's LDS buffers (a static
// LDS variable would shift the dynamic buffers off their 16-byte alignment,
// which ran three times slower).
template <int WPW, int SUB, int CHUNK, int OCC, bool PIPE, int DEPTH, int NW>
__global__ void __launch_bounds__(64 * NW, OCC) k_chi0_bf16x3_persistent(const TileQueue *q) {
  typedef Cfg<WPW, SUB, CHUNK, NW> C;
  extern __shared__ unsigned int lds[];
  int *next_tile = (int *)(lds + variant_lds<WPW, SUB, CHUNK, PIPE, DEPTH, NW>() / 4);
  for (;;) {
    if (threadIdx.x == 0) *next_tile = atomicAdd(&q->counter[0], 1);
    __syncthreads();
    const int idx = *next_tile;
    if (idx >= q->n_tiles) break;
    const BatchTile tl = q->tiles[idx];
    const BatchItem it = q->items[tl.item];
    const long long t_lo = tl.slice * it.slice_len;
    const long long t_hi = std::min(it.n_trans, t_lo + it.slice_len);
    const int col0 = tl.gc * C::kCols;
    if (tl.gb < 0) {
      // a tail tile: wblk counts groups of 16 WPW NW virtual rows
      const TailGeom tg{it.nm, it.tail, tl.wblk * 16 * WPW * NW,
                        it.tpart + (size_t)tl.slice * it.n_w * it.tail * 2 * it.ld};
      run_tail_tile<WPW, SUB, CHUNK, PIPE, DEPTH, NW>(std::min(SUB, (it.ld - col0) / 16), lds, it.P,
                                                      it.R, it.ld, it.delta, it.df, it.n_trans,
                                                      t_lo, t_hi, it.omega, it.n_w, it.eta,
                                                      it.paired, it.n_g, col0, tg);
    } else {
      run_tile<WPW, SUB, CHUNK, PIPE, DEPTH, NW>(std::min(SUB, (it.lc - col0) / 16), lds, it.P, it.R,
                                                 it.ld, it.delta, it.df, it.n_trans, t_lo, t_hi,
                                                 it.omega, it.n_w, it.eta, it.paired, it.n_g,
                                                 tl.wblk * C::kWBlock, tl.gb * 16, col0,
                                                 it.part + (size_t)tl.slice * it.n_w * it.n_g * it.n_g);
    }
    // the next tile's prologue rewrites the LDS buffers, and thread 0 the
    // tile index every thread has read
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&q->counter[1], 1) == (int)gridDim.x - 1) {
      atomicExch(&q->counter[0], 0);
      atomicExch(&q->counter[1], 0);
    }
  }
}

struct Variant {
  int wpw, sub, chunk, occ, waves;
  bool pipe;
  size_t lds;
  const void *grid_fn;
  const void *pers_fn;
};

#define TDX_V(W, S, K, O, PIPE, DEPTH, NW)                                               \
  Variant {                                                                              \
    W, S, K, O, NW, PIPE, variant_lds<W, S, K, PIPE, DEPTH, NW>(),                       \
        (const void *)k_chi0_bf16x3<W, S, K, O, PIPE, DEPTH, NW>,                        \
        (const void *)k_chi0_bf16x3_persistent<W, S, K, O, PIPE, DEPTH, NW>              \
  }
const Variant kVariants[] = {TDX_V(4, 4, 32, 2, false, 2, 4), TDX_V(2, 8, 16, 2, false, 2, 4),
                             TDX_V(4, 2, 32, 2, false, 2, 4), TDX_V(2, 4, 32, 2, false, 2, 4),
                             TDX_V(2, 9, 16, 2, false, 2, 4), TDX_V(2, 8, 32, 2, false, 2, 4),
                             TDX_V(2, 9, 32, 1, true, 0, 4),  TDX_V(2, 9, 16, 2, false, 3, 4),
                             TDX_V(2, 9, 32, 1, false, 2, 8), TDX_V(2, 9, 32, 1, false, 3, 8),
                             TDX_V(1, 9, 32, 1, true, 0, 12)};
#undef TDX_V

}  // namespace

int bf16x3_variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }

int bf16x3_default_variant() { return 9; }  // TDX_V(2, 9, 32, 1, false, 3, 8)

void bf16x3_variant_shape(int v, int *wblock, int *cols) {
  *wblock = kVariants[v].waves * kVariants[v].wpw;
  *cols = 16 * kVariants[v].sub;
}

int bf16x3_variant_occupancy(int v) { return kVariants[v].occ; }

TailSplit bf16x3_split(int v, int n_g) {
  const int ld = (n_g + 15) / 16 * 16;
  if (kVariants[v].pipe) return TailSplit{ld, 0};
  if (n_g % 16 != 0) return TailSplit{n_g / 16 * 16, n_g % 16};
  // a whole last block that would make a main column tile of its own (the
  // 16-proton basis, N_G = 304: 19 blocks as 9 + 9 + 1) runs as 16 tail
  // rows instead, so the main tiles keep full width
  const int blocks = n_g / 16;
  if (blocks > 1 && blocks % kVariants[v].sub == 1) return TailSplit{n_g - 16, 16};
  return TailSplit{ld, 0};
}

int bf16x3_tail_groups(int v, int n_w, int tail) {
  const int rows = 16 * kVariants[v].wpw * kVariants[v].waves;
  return tail > 0 ? (n_w * 2 * tail + rows - 1) / rows : 0;
}

int bf16x3_launch_grid(int v, const void *P, const void *R, int ld, const double *delta,
                       const double *df,
                       long long n_trans, long long slice_len, int slices, const double *omega,
                       int n_w, double eta, int paired, int n_g, double2 *part, double2 *tpart,
                       hipStream_t s) {
  const Variant &V = kVariants[v];
  const TailSplit sp = bf16x3_split(v, n_g);
  int lc = sp.nm, nm = sp.nm, tail = sp.tail;
  const int wb = V.waves * V.wpw;
  int ncb = (lc + 16 * V.sub - 1) / (16 * V.sub);
  int nx = (n_w + wb - 1) / wb, ny = (lc / 16) * ncb;
  int ntg = bf16x3_tail_groups(v, n_w, tail), nct = (ld + 16 * V.sub - 1) / (16 * V.sub);
  int n_tail = tail > 0 ? ntg * nct * slices : 0;
  const long long total = (long long)n_tail + (long long)nx * ny * slices;
  TDX_REQUIRE(total > 0 && total < (1LL << 31), TDX_ERR_SHAPE, "%lld tiles", total);
  TDX_HIP(hipFuncSetAttribute(V.grid_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)V.lds));
  void *args[] = {(void *)&P,       (void *)&R,         (void *)&ld,    (void *)&delta,
                  (void *)&df,      (void *)&n_trans,   (void *)&slice_len,
                  (void *)&omega,   (void *)&n_w,       (void *)&eta,   (void *)&paired,
                  (void *)&n_g,     (void *)&lc,        (void *)&nx,    (void *)&ncb,
                  (void *)&ny,      (void *)&n_tail,    (void *)&ntg,   (void *)&nct,
                  (void *)&nm,      (void *)&tail,      (void *)&part,  (void *)&tpart};
  TDX_HIP(hipLaunchKernel(V.grid_fn, dim3((unsigned)total), dim3(64 * V.waves), args, V.lds, s));
  return TDX_OK;
}

int bf16x3_launch_persistent(int v, const TileQueue *queue, int n_blocks, hipStream_t s) {
  const Variant &V = kVariants[v];
  const size_t lds = V.lds + 16;  // the tile-index word after the buffers
  TDX_HIP(hipFuncSetAttribute(V.pers_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  void *args[] = {(void *)&queue};
  TDX_HIP(hipLaunchKernel(V.pers_fn, dim3(n_blocks), dim3(64 * V.waves), args, lds, s));
  return TDX_OK;
}

}  // namespace tdx
