// Work descriptors shared by the chi0 launch forms (internal).
#pragma once

#include <hip/hip_runtime.h>

namespace tdx {

// One q-vector of a batch: its transitions, pair densities and outputs.
struct BatchItem {
  const void *P;  // split-BF16 fragment words
  const void *R;  // FP32 rho rows that follow them
  int ld;
  const double *delta, *df;
  long long n_trans, slice_len;
  const double *omega;
  int n_w;
  double eta;
  int paired;  // time-reversal paired transition list
  int n_g;
  double2 *part;  // [slices][n_w][n_g][n_g]
  int lc;         // rows and columns of the main tiles (ld, or nm with tail tiles)
  int nm, tail;   // tail tiles: basis rows nm .. nm + tail - 1 (tail = 0: none)
  double2 *tpart; // [slices][n_w][tail][2][ld]
};

// One tile of the work queue; gb < 0 marks a tail tile whose wblk counts
// groups of virtual rows.
struct BatchTile {
  int item, wblk, gb, gc;
  long long slice;
};

// The persistent kernel's work, in device memory: the tile list, its items
// and two counter words (next tile, workgroups done), zero before the first
// launch and left zero by every launch.
struct TileQueue {
  const BatchItem *items;
  const BatchTile *tiles;
  int n_tiles;
  int *counter;
};

// Rows and columns [0, nm) of a basis run in main tiles, rows nm .. n_g - 1
// (tail of them, at most 16) in tail tiles.  nm = 16 floor(n_g / 16) when
// n_g is not a multiple of 16; for a multiple of 16, nm = n_g - 16 and
// tail = 16 when the last block would otherwise be a main column tile of
// its own, else nm = ld and tail = 0; a pipelined variant has no tail.
struct TailSplit {
  int nm, tail;
};
TailSplit bf16x3_split(int v, int n_g);
// Workgroups of virtual tail rows (2 tail per frequency) for n_w frequencies.
int bf16x3_tail_groups(int v, int n_w, int tail);

int bf16x3_variant_count();
// Variant used for a basis size with no tuned entry: the 8-wave 2 x 9 tile
// with three LDS buffers, the fastest variant measured on every basis size
// tried (N_G 133 to 303).
int bf16x3_default_variant();
void bf16x3_variant_shape(int v, int *wblock, int *cols);
int bf16x3_variant_occupancy(int v);  // workgroups per CU
// The FP32 rho block that follows the fragment words of a split-BF16
// pair-density buffer laid out for p_rows transitions (rows padded to a
// multiple of 32 plus one zero chunk of 32).
inline const void *bf16x3_rho(const void *P, long long p_rows, int ld) {
  return (const char *)P + (size_t)(((p_rows + 31) / 32 + 1) * 32) * ld * 8;
}

int bf16x3_launch_grid(int v, const void *P, const void *R, int ld, const double *delta,
                       const double *df,
                       long long n_trans, long long slice_len, int slices, const double *omega,
                       int n_w, double eta, int paired, int n_g, double2 *part, double2 *tpart,
                       hipStream_t s);
int bf16x3_launch_persistent(int v, const TileQueue *queue, int n_blocks, hipStream_t s);

}  // namespace tdx
