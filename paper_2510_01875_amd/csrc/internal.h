// Internal declarations shared by the tdx library sources (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/tdx.h"

namespace tdx {

// ---------------------------------------------------------------- errors
int fail(int code, const char *fmt, ...);
void clear_error();

#define TDX_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      return ::tdx::fail(TDX_ERR_HIP, "%s failed: %s (%s:%d)", #call,        \
                         hipGetErrorString(e_), __FILE__, __LINE__);         \
  } while (0)

#define TDX_REQUIRE(cond, code, ...)                                         \
  do {                                                                       \
    if (!(cond)) return ::tdx::fail(code, __VA_ARGS__);                      \
  } while (0)

#define TDX_TRY(expr)                                                        \
  do {                                                                       \
    int r_ = (expr);                                                         \
    if (r_ != TDX_OK) return r_;                                             \
  } while (0)

// ------------------------------------------------------------- workspace
// Named, grow-only device buffers owned by the context.
struct Workspace {
  void *ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace tdx

// Tile variant and slice length of a chi0 kernel for one precision and
// response-basis size class (ld / 16 blocks); variant -1 = default.  The
// FP32 and FP64 kernels choose their slices to fill the chip and use only
// the variant.
struct tdx_chi0_tune {
  int variant = -1;  // -1: the default variant
  int slice_log2 = 20;
  double ms = 0.0;
};

struct tdx_ctx {
  int device = 0;
  int n_cu = 0;
  rocblas_handle blas = nullptr;
  size_t limit = 0;  // 0 = unlimited
  tdx::Workspace ws[13];
  tdx_chi0_tune tune[3][64];  // [prec][size class]
  long long slice_len = 0;  // chi0 slice length; 0 = chosen per call to fill the chip
};

namespace tdx {

enum WsSlot {
  WS_EIG = 0,      // Hamiltonians / eigenvectors for a batch of k
  WS_EIG_AUX = 1,  // eigenvalues, tridiagonal scratch, info
  WS_ROWS = 2,     // per-row transition counts
  WS_PARTIAL = 3,  // chi0 split-K partial sums
  WS_DYSON = 4,    // Dyson matrices
  WS_DENS = 5,     // density partial sums
  WS_MISC = 6,     // small per-call tables (k+q maps, lookups)
  WS_MISC2 = 7,
  WS_ADJ = 8,       // adjoint: per-frequency vectors, state tables
  WS_ADJ2 = 9,      // adjoint: eigen-adjoint products
  WS_ADJ3 = 10,     // adjoint: reductions
  WS_FXC = 11,      // f_xc(G) grid of the composed kernel-matrix call
  WS_SG = 12,       // window and degree lists of a Savitzky-Golay filter bank
};

size_t ws_total(const tdx_ctx *ctx);
// Ensure slot holds at least `bytes`; respects ctx->limit.
int ws_get(tdx_ctx *ctx, int slot, size_t bytes, void **out);

inline hipStream_t as_stream(tdx_stream s) { return reinterpret_cast<hipStream_t>(s); }

// ------------------------------------------------------------- geometry
struct Lattice {
  double a[3][3];   // rows a_i
  double b[3][3];   // rows b_i, a_i . b_j = 2 pi delta_ij
  double volume;
};

int make_lattice(const double cell[9], Lattice *L);

// Monkhorst-Pack point r (multi-index) in reduced coordinates.
inline void mp_point(const int N[3], int r0, int r1, int r2, double red[3]) {
  const int r[3] = {r0, r1, r2};
  for (int i = 0; i < 3; ++i) red[i] = (2.0 * r[i] + 1.0 - N[i]) / (2.0 * N[i]);
}

inline void kindex_split(int k, const int N[3], int r[3]) {
  r[2] = k % N[2];
  r[1] = (k / N[2]) % N[1];
  r[0] = k / (N[1] * N[2]);
}

// k_r + q = k_{r'} + G_s for q = sum qj_i/N_i b_i.
void kq_map(const int N[3], const int qj[3], std::vector<int> *kp, std::vector<int> *gs);

// Plane-wave sphere 1/2|k+G|^2 <= ecut, sorted by |k+G|^2 then Miller.
void gsphere(const Lattice &L, const double kred[3], double ecut, std::vector<int> *m);

int check_device(tdx_ctx *ctx);

// Resolves the device address of the no-allocation Dyson scratch for
// `device` (which must be current); called by tdx_create.
int dyson_scratch_init(int device);

}  // namespace tdx
