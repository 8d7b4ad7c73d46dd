// Work descriptors shared by the chi0 launch forms (internal).
#pragma once

#include <hip/hip_runtime.h>

namespace tdx {

// One q-vector of a batch: its transitions, pair densities and outputs.
struct BatchItem {
  const void *P;
  int ld;
  const double *delta, *df;
  long long n_trans, slice_len;
  const double *omega;
  int n_w;
  double eta;
  int n_g;
  double2 *part;  // [slices][n_w][n_g][n_g]
};

// One tile of the work queue.
struct BatchTile {
  int item, wblk, gb, gc;
  long long slice;
};

int bf16x3_variant_count();
void bf16x3_variant_shape(int v, int *wblock, int *cols);
int bf16x3_launch_grid(int v, const void *P, int ld, const double *delta, const double *df,
                       long long n_trans, long long slice_len, int slices, const double *omega,
                       int n_w, double eta, int n_g, double2 *part, hipStream_t s);
int bf16x3_launch_persistent(int v, const BatchItem *items, const BatchTile *tiles, int n_tiles,
                             int n_blocks, hipStream_t s);

}  // namespace tdx
