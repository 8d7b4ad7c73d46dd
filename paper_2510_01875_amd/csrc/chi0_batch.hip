// Split-BF16 chi0 drivers: single q (grid launch), ragged batches of q in
// one persistent launch (a plan whose launch is free of allocation, host
// synchronisation and memset, so it can be captured in a HIP graph), the
// slice reduction, and the tile/slice autotuner with its on-disk cache.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <vector>

#include "chi0_batch.h"
#include "internal.h"

namespace tdx {

int chi0_fp_variant_count(bool f64);  // chi0_fp.hip

namespace {

constexpr int kChunkAlign = 32;   // slice lengths are multiples of every variant's chunk
constexpr int kMinTiles = 2048;   // fill the chip: 256 CUs x 2 workgroups x 4

// The slice reduction of one q: chi0[w][G][G'] = pref sum over slices, in
// slice order, of the main partials (G, G' < nm) or, with tail tiles, of the
// tail rows of H_R and H_A: rows G >= nm are H_R + i H_A of the tail row
// G - nm, columns G' >= nm (G < nm) are conj(H_R) + i conj(H_A) of the tail
// row G' - nm at column G (H_R and H_A are Hermitian).
struct ReduceItem {
  const double2 *part;
  int n_slices;
  int n_w, n_g, nm, tail, ld;
  double pref;
  const double2 *tpart;
  double2 *out;
};

__device__ inline void reduce_one(const ReduceItem &it, size_t i) {
  const size_t per = (size_t)it.n_w * it.n_g * it.n_g;
  const size_t tper = (size_t)it.n_w * it.tail * 2 * it.ld;
  const int w = (int)(i / ((size_t)it.n_g * it.n_g));
  const int rem = (int)(i % ((size_t)it.n_g * it.n_g));
  const int G = rem / it.n_g, Gp = rem % it.n_g;
  double re = 0.0, im = 0.0;
  if (it.tail == 0 || (G < it.nm && Gp < it.nm)) {
    for (int s = 0; s < it.n_slices; ++s) {
      const double2 v = it.part[(size_t)s * per + i];
      re += v.x;
      im += v.y;
    }
  } else {
    const bool row = G >= it.nm;
    const int g = row ? G - it.nm : Gp - it.nm, col = row ? Gp : G;
    const size_t o = (((size_t)w * it.tail + g) * 2) * it.ld + col;
    for (int s = 0; s < it.n_slices; ++s) {
      const double2 hr = it.tpart[(size_t)s * tper + o];
      const double2 ha = it.tpart[(size_t)s * tper + o + it.ld];
      re += row ? hr.x - ha.y : hr.x + ha.y;
      im += row ? hr.y + ha.x : ha.x - hr.y;
    }
  }
  it.out[i] = make_double2(it.pref * re, it.pref * im);
}

__global__ void k_reduce_slices(ReduceItem it) {
  const size_t n = (size_t)it.n_w * it.n_g * it.n_g;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    reduce_one(it, i);
}

// Slice reduction of every item of a batch (blockIdx.y = item).
__global__ void k_reduce_batch(const ReduceItem *items) {
  const ReduceItem it = items[blockIdx.y];
  const size_t n = (size_t)it.n_w * it.n_g * it.n_g;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    reduce_one(it, i);
}

int bucket_of(int ld) { return std::min(ld / 16, 63); }

void pick(const tdx_ctx *ctx, int ld, int *variant, int *slice_log2) {
  const tdx_chi0_tune &t = ctx->tune[TDX_PREC_BF16X3][bucket_of(ld)];
  *variant = t.variant >= 0 ? t.variant : bf16x3_default_variant();
  *slice_log2 = t.slice_log2;
}

// Tile variants of a precision (the FP32 and FP64 ones in chi0_fp.hip).
int variant_count(int prec) {
  return prec == TDX_PREC_BF16X3 ? bf16x3_variant_count()
                                 : chi0_fp_variant_count(prec == TDX_PREC_FP64);
}

const char *prec_name(int prec) {
  return prec == TDX_PREC_FP64 ? "fp64" : prec == TDX_PREC_FP32 ? "fp32" : "bf16x3";
}

// Tiles of one slice for the round model below: main tiles (one row block,
// column tile and frequency block each) and tail tiles, and the cost of a
// tail tile relative to a main one (its column blocks over the main tile's,
// and about a fifth more for the weights each lane forms itself).
struct SliceTiles {
  long long main, tail;
  double tail_cost;
};
SliceTiles slice_tiles(int v, int n_w, int n_g);

// Fixed cost of a tile (prologue and fold) in transition-equivalents.
constexpr double kTileFixed = 1024.0;

long long chunk_len(long long n_trans, long long ns) {
  const long long len = (n_trans + ns - 1) / ns;
  return (len + kChunkAlign - 1) / kChunkAlign * kChunkAlign;
}

// Tile costs of a list cut into slices of len transitions, as (cost, count)
// groups: a tile costs its slice's transitions plus kTileFixed, times
// tail_cost for a tail tile.
void add_tile_groups(std::vector<std::pair<double, long long>> &g, long long n_trans,
                     long long len, const SliceTiles &t) {
  const long long ns = (n_trans + len - 1) / len, last = n_trans - (ns - 1) * len;
  const double full = (double)len + kTileFixed, part = (double)last + kTileFixed;
  g.push_back({full * t.tail_cost, (ns - 1) * t.tail});
  g.push_back({part * t.tail_cost, t.tail});
  g.push_back({full, (ns - 1) * t.main});
  g.push_back({part, t.main});
}

// Predicted end of a queue of tiles on `slots` workgroup slots, each tile
// starting on the slot that frees first, the costliest first.  Tiles of one
// cost fill the slots level by level, so the slots are kept as groups of
// equal finishing time.
double makespan(std::vector<std::pair<double, long long>> g, int slots) {
  std::sort(g.begin(), g.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
  std::map<double, long long> at;  // finishing time -> slots
  at[0.0] = slots;
  for (const auto &x : g) {
    long long count = x.second;
    while (count > 0) {
      auto it = at.begin();
      const double t0 = it->first;
      const long long m = it->second, k = std::min(m, count);
      if (k == m)
        at.erase(it);
      else
        it->second = m - k;
      at[t0 + x.first] += k;
      count -= k;
    }
  }
  return at.rbegin()->first;
}

// Slice counts allowed for a list: from the minimum, about 2^slice_log2
// transitions a slice but at least enough tiles to fill the chip, up to 4
// times that, with the slice partials held within 4 times the minimum's or
// 16 GiB, whichever is larger than the minimum's own.
struct SliceRange {
  long long ns0, ns_hi;
};
SliceRange slice_range(long long n_trans, int slice_log2, const SliceTiles &tiles,
                       size_t bytes_per_slice) {
  const long long tps = std::max<long long>(1, tiles.main + tiles.tail);
  const long long ns_cap = std::max<long long>(
      1, std::min<long long>((n_trans + kChunkAlign - 1) / kChunkAlign, 8192));
  long long ns0 = std::max<long long>((n_trans + (1LL << slice_log2) - 1) >> slice_log2,
                                      (kMinTiles + tps - 1) / tps);
  ns0 = std::max<long long>(1, std::min<long long>(ns0, ns_cap));
  const size_t cap_bytes = std::max<size_t>(
      (size_t)ns0 * bytes_per_slice, std::min<size_t>(4 * ns0 * bytes_per_slice, (size_t)16 << 30));
  long long ns_hi = std::min<long long>(4 * ns0, ns_cap);
  if (bytes_per_slice > 0)
    ns_hi = std::min<long long>(ns_hi, (long long)(cap_bytes / bytes_per_slice));
  return SliceRange{ns0, std::max(ns_hi, ns0)};
}

// Slices of a transition list, a multiple of the chunk long; with a fixed
// length set on the context, slices of that length.  Tiles run in rounds of
// one per workgroup slot, so a count just past a whole number of rounds
// leaves most of the chip idle in the last one (the crystal's N_G = 129
// basis: 8 slices of 260 tiles on 256 slots are 8.1 rounds); the slice
// count in slice_range that minimises the makespan is taken, the fewest
// within 0.5 % of the best.  Lists of many rounds keep the minimum, whose
// last round is a small share.
void slicing_fixed(long long fixed_len, long long n_trans, int slice_log2,
                   const SliceTiles &tiles, int slots, size_t bytes_per_slice,
                   long long *slice_len, int *slices) {
  long long len;
  if (fixed_len > 0) {
    len = (fixed_len + kChunkAlign - 1) / kChunkAlign * kChunkAlign;
  } else {
    const SliceRange r = slice_range(n_trans, slice_log2, tiles, bytes_per_slice);
    long long best_ns = r.ns0;
    if (slots > 0 && r.ns0 * (tiles.main + tiles.tail) < 64LL * slots) {
      std::vector<std::pair<long long, double>> cand;
      double best = 1e300;
      for (long long ns = r.ns0; ns <= r.ns_hi; ++ns) {
        if (ns > r.ns0 && chunk_len(n_trans, ns) == chunk_len(n_trans, ns - 1)) continue;
        std::vector<std::pair<double, long long>> g;
        add_tile_groups(g, n_trans, chunk_len(n_trans, ns), tiles);
        const double t = makespan(g, slots);
        cand.push_back({ns, t});
        best = std::min(best, t);
      }
      for (const auto &c : cand)
        if (c.second <= 1.005 * best) {
          best_ns = c.first;
          break;
        }
    }
    len = chunk_len(n_trans, best_ns);
  }
  *slice_len = len;
  *slices = (int)std::max<long long>(1, (n_trans + len - 1) / len);
}

void slicing(const tdx_ctx *ctx, long long n_trans, int slice_log2, const SliceTiles &tiles,
             int slots, size_t bytes_per_slice, long long *slice_len, int *slices) {
  slicing_fixed(ctx->slice_len, n_trans, slice_log2, tiles, slots, bytes_per_slice, slice_len,
                slices);
}

SliceTiles slice_tiles(int v, int n_w, int n_g) {
  int wb, cols;
  bf16x3_variant_shape(v, &wb, &cols);
  const int ld = (n_g + 15) / 16 * 16;
  const TailSplit sp = bf16x3_split(v, n_g);
  SliceTiles t;
  t.main = (long long)((n_w + wb - 1) / wb) * (sp.nm / 16) * ((sp.nm + cols - 1) / cols);
  t.tail = (long long)bf16x3_tail_groups(v, n_w, sp.tail) * ((ld + cols - 1) / cols);
  const int main_blocks = std::min(sp.nm / 16, cols / 16), tail_blocks = std::min(ld / 16, cols / 16);
  t.tail_cost = main_blocks > 0 ? 1.2 * tail_blocks / main_blocks : 1.2;
  return t;
}

}  // namespace

int chi0_bf16x3_with(tdx_ctx *ctx, int v, int slice_log2, const void *P, long long p_rows,
                     int ld, const double *delta, const double *df, int paired,
                     long long n_trans, const double *omega, int n_w, double eta, int n_g,
                     double pref, double2 *chi0, hipStream_t s) {
  long long slice_len;
  int slices;
  const TailSplit sp = bf16x3_split(v, n_g);
  const size_t out_elems = (size_t)n_w * n_g * n_g;
  const size_t tail_elems = (size_t)n_w * sp.tail * 2 * ld;
  slicing(ctx, n_trans, slice_log2, slice_tiles(v, n_w, n_g),
          bf16x3_variant_occupancy(v) * std::max(ctx->n_cu, 1),
          sizeof(double2) * (out_elems + tail_elems), &slice_len, &slices);
  TDX_REQUIRE(slices <= 65535, TDX_ERR_SHAPE, "%d slices exceed the grid (slice length %lld)",
              slices, slice_len);
  void *w;
  TDX_TRY(ws_get(ctx, WS_PARTIAL, sizeof(double2) * (out_elems + tail_elems) * slices, &w));
  double2 *part = (double2 *)w;
  double2 *tpart = part + out_elems * slices;
  TDX_TRY(bf16x3_launch_grid(v, P, bf16x3_rho(P, p_rows, ld), ld, delta, df, n_trans, slice_len,
                             slices, omega, n_w, eta, paired, n_g, part, tpart, s));
  const unsigned rb = (unsigned)std::min<size_t>((out_elems + 255) / 256, 8192);
  const ReduceItem ri{part, slices, n_w, n_g, sp.nm, sp.tail, ld, pref, tpart, chi0};
  hipLaunchKernelGGL(k_reduce_slices, dim3(rb), dim3(256), 0, s, ri);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

int chi0_bf16x3(tdx_ctx *ctx, const void *P, int ld, const double *delta, const double *df,
                int paired, long long n_trans, const double *omega, int n_w, double eta, int n_g,
                double pref, double2 *chi0, hipStream_t s) {
  int v, sl;
  pick(ctx, ld, &v, &sl);
  return chi0_bf16x3_with(ctx, v, sl, P, n_trans, ld, delta, df, paired, n_trans, omega, n_w,
                          eta, n_g, pref, chi0, s);
}

}  // namespace tdx

// ------------------------------------------------------------------ plans
struct tdx_chi0_plan {
  int device = 0;
  int prec = 0;
  int variant = 0;
  int n_items = 0, n_tiles = 0, n_blocks = 0;
  void *mem = nullptr;  // one device allocation for everything below
  tdx::BatchItem *items = nullptr;
  tdx::BatchTile *tiles = nullptr;
  tdx::ReduceItem *reduce = nullptr;
  int *counter = nullptr;
  tdx::TileQueue *queue = nullptr;
  size_t max_per_slice = 0;
  std::vector<tdx_chi0_item> host_items;  // for the non-persistent precisions
};

using namespace tdx;

extern "C" {

int tdx_chi0_variants(int prec, int *count) {
  clear_error();
  TDX_REQUIRE(count, TDX_ERR_INVALID_ARG, "count is null");
  TDX_REQUIRE(prec >= TDX_PREC_FP64 && prec <= TDX_PREC_BF16X3, TDX_ERR_INVALID_ARG, "bad prec");
  *count = variant_count(prec);
  return TDX_OK;
}

int tdx_chi0_set_config(tdx_ctx *ctx, int prec, int n_g, int variant, int slice_log2) {
  clear_error();
  TDX_REQUIRE(ctx, TDX_ERR_INVALID_ARG, "ctx is null");
  TDX_REQUIRE(prec >= TDX_PREC_FP64 && prec <= TDX_PREC_BF16X3, TDX_ERR_INVALID_ARG, "bad prec");
  TDX_REQUIRE(variant >= -1 && variant < variant_count(prec), TDX_ERR_INVALID_ARG,
              "bad variant %d", variant);
  TDX_REQUIRE(slice_log2 >= 10 && slice_log2 <= 30, TDX_ERR_INVALID_ARG, "bad slice_log2");
  TDX_REQUIRE(n_g > 0, TDX_ERR_INVALID_ARG, "bad n_g");
  tdx_chi0_tune &t = ctx->tune[prec][bucket_of((n_g + 15) / 16 * 16)];
  t.variant = variant;
  t.slice_log2 = slice_log2;
  return TDX_OK;
}

int tdx_chi0_set_slice_length(tdx_ctx *ctx, int64_t n) {
  clear_error();
  TDX_REQUIRE(ctx, TDX_ERR_INVALID_ARG, "ctx is null");
  TDX_REQUIRE(n >= 0 && n <= (1LL << 40), TDX_ERR_INVALID_ARG, "bad slice length %lld",
              (long long)n);
  ctx->slice_len = (long long)n;
  return TDX_OK;
}

int tdx_chi0_bf16x3_slicing(int n_cu, int variant, int64_t n_trans, int n_g, int n_w,
                            int slice_log2, int64_t *slice_len, int *slices) {
  clear_error();
  TDX_REQUIRE(slice_len && slices, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_cu > 0 && n_trans > 0 && n_g > 0 && n_w > 0, TDX_ERR_INVALID_ARG,
              "bad sizes (n_cu %d, n_trans %lld, n_g %d, n_w %d)", n_cu, (long long)n_trans, n_g,
              n_w);
  TDX_REQUIRE(variant >= 0 && variant < bf16x3_variant_count(), TDX_ERR_INVALID_ARG,
              "bad variant %d", variant);
  TDX_REQUIRE(slice_log2 >= 10 && slice_log2 <= 30, TDX_ERR_INVALID_ARG, "bad slice_log2");
  const int ld = (n_g + 15) / 16 * 16;
  const TailSplit sp = bf16x3_split(variant, n_g);
  long long len;
  int ns;
  slicing_fixed(0, n_trans, slice_log2, slice_tiles(variant, n_w, n_g),
                bf16x3_variant_occupancy(variant) * n_cu,
                sizeof(double2) * ((size_t)n_w * n_g * n_g + (size_t)n_w * sp.tail * 2 * ld),
                &len, &ns);
  *slice_len = len;
  *slices = ns;
  return TDX_OK;
}

int tdx_chi0_get_config(tdx_ctx *ctx, int prec, int n_g, int *variant, int *slice_log2) {
  clear_error();
  TDX_REQUIRE(ctx && variant && slice_log2, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(prec >= TDX_PREC_FP64 && prec <= TDX_PREC_BF16X3, TDX_ERR_INVALID_ARG, "bad prec");
  if (prec == TDX_PREC_BF16X3) {
    pick(ctx, (n_g + 15) / 16 * 16, variant, slice_log2);
  } else {
    const tdx_chi0_tune &t = ctx->tune[prec][bucket_of((n_g + 15) / 16 * 16)];
    *variant = t.variant >= 0 ? t.variant : 0;
    *slice_log2 = t.slice_log2;
  }
  return TDX_OK;
}

int tdx_chi0_plan_create(tdx_ctx *ctx, const tdx_chi0_item *items, int n_items, int prec,
                         tdx_chi0_plan **out) {
  clear_error();
  TDX_REQUIRE(ctx && items && out && n_items > 0, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(prec >= TDX_PREC_FP64 && prec <= TDX_PREC_BF16X3, TDX_ERR_INVALID_ARG, "bad prec");
  for (int i = 0; i < n_items; ++i) {
    const tdx_chi0_item &it = items[i];
    TDX_REQUIRE(it.tl && it.P && it.omega && it.chi0, TDX_ERR_INVALID_ARG,
                "item %d has a null pointer", i);
    TDX_REQUIRE(it.n_g > 0 && it.n_w > 0 && it.n_trans > 0 && it.n_trans <= it.tl->capacity &&
                    it.p_rows >= 0 && (it.p_rows == 0 || it.n_trans <= it.p_rows),
                TDX_ERR_SHAPE, "item %d has bad sizes", i);
    TDX_REQUIRE(std::isfinite(it.eta) && it.eta > 0 && std::isfinite(it.pref),
                TDX_ERR_INVALID_ARG, "item %d has a bad eta or prefactor", i);
  }
  TDX_TRY(check_device(ctx));
  tdx_chi0_plan *p = new tdx_chi0_plan();
  p->device = ctx->device;
  p->prec = prec;
  p->n_items = n_items;
  p->host_items.assign(items, items + n_items);
  if (prec != TDX_PREC_BF16X3) {
    *out = p;
    return TDX_OK;
  }
  // one tile variant for the whole launch: the configuration of the widest basis
  int ld_max = 0;
  for (int i = 0; i < n_items; ++i) ld_max = std::max(ld_max, (items[i].n_g + 15) / 16 * 16);
  int v, sl_default;
  pick(ctx, ld_max, &v, &sl_default);
  p->variant = v;
  int wb, cols;
  bf16x3_variant_shape(v, &wb, &cols);
  // slice counts: each list as a grid launch of it would slice it, so the
  // plan's results are bitwise those of one launch per list
  const int slots = bf16x3_variant_occupancy(v) * std::max(ctx->n_cu, 1);
  std::vector<long long> slen(n_items);
  std::vector<SliceTiles> stiles(n_items);
  for (int i = 0; i < n_items; ++i) {
    const tdx_chi0_item &it = items[i];
    const int ld = (it.n_g + 15) / 16 * 16;
    int vi, sl;
    pick(ctx, ld, &vi, &sl);
    const TailSplit sp = bf16x3_split(v, it.n_g);
    stiles[i] = slice_tiles(v, it.n_w, it.n_g);
    const size_t bytes = sizeof(double2) * ((size_t)it.n_w * it.n_g * it.n_g +
                                            (size_t)it.n_w * sp.tail * 2 * ld);
    int ns;
    slicing(ctx, it.n_trans, sl, stiles[i], slots, bytes, &slen[i], &ns);
  }
  std::vector<BatchItem> bi(n_items);
  std::vector<ReduceItem> ri(n_items);
  std::vector<BatchTile> tiles;
  size_t part_bytes = 0;
  std::vector<size_t> part_off(n_items);
  for (int i = 0; i < n_items; ++i) {
    const tdx_chi0_item &it = items[i];
    const int ld = (it.n_g + 15) / 16 * 16;
    const TailSplit sp = bf16x3_split(v, it.n_g);
    const long long slice_len = slen[i];
    const int slices = (int)((it.n_trans + slice_len - 1) / slice_len);
    const size_t per = (size_t)it.n_w * it.n_g * it.n_g;
    const size_t tper = (size_t)it.n_w * sp.tail * 2 * ld;
    part_off[i] = part_bytes;
    part_bytes += (per + tper) * slices * sizeof(double2);
    p->max_per_slice = std::max(p->max_per_slice, per);
    // the FP32 rows follow the fragment words of all p_rows transitions the
    // buffer was written for, of which the first n_trans are contracted
    const long long rows = it.p_rows > 0 ? it.p_rows : it.n_trans;
    bi[i] = BatchItem{it.P,        bf16x3_rho(it.P, rows, ld), ld, it.tl->delta,
                      it.tl->df,   (long long)it.n_trans, slice_len, it.omega,
                      it.n_w,      it.eta,      (int)it.tl->paired,   it.n_g,
                      nullptr,     sp.nm,       sp.nm,        sp.tail,
                      nullptr};
    ri[i] = ReduceItem{nullptr, slices, it.n_w, it.n_g, sp.nm, sp.tail, ld, it.pref, nullptr,
                       (double2 *)it.chi0};
    const int nwb = (it.n_w + wb - 1) / wb, ngb = sp.nm / 16, ncb = (sp.nm + cols - 1) / cols;
    // tail tiles (gb = -1) first, as they hold the most column blocks:
    // groups of virtual rows over every column tile
    const int ntg = bf16x3_tail_groups(v, it.n_w, sp.tail), nct = (ld + cols - 1) / cols;
    for (int s = 0; s < slices; ++s)
      for (int c = 0; c < nct; ++c)
        for (int a = 0; a < ntg; ++a) tiles.push_back(BatchTile{i, a, -1, c, s});
    // frequency block fastest: consecutive tiles read the same rho rows
    for (int s = 0; s < slices; ++s)
      for (int g = 0; g < ngb; ++g)
        for (int c = 0; c < ncb; ++c)
          for (int a = 0; a < nwb; ++a) tiles.push_back(BatchTile{i, a, g, c, s});
  }
  // costliest tiles first (tail tiles hold more column blocks, the last
  // slice of an item is shorter)
  std::stable_sort(tiles.begin(), tiles.end(), [&](const BatchTile &a, const BatchTile &b) {
    auto cost = [&](const BatchTile &t) {
      const BatchItem &x = bi[t.item];
      const double len = (double)std::min(x.slice_len, x.n_trans - t.slice * x.slice_len);
      return (len + kTileFixed) * (t.gb < 0 ? stiles[t.item].tail_cost : 1.0);
    };
    return cost(a) > cost(b);
  });
  TDX_REQUIRE(tiles.size() < (size_t)1 << 30, TDX_ERR_SHAPE, "too many tiles");
  const size_t off_items = (part_bytes + 255) / 256 * 256;
  const size_t off_reduce = off_items + (sizeof(BatchItem) * n_items + 255) / 256 * 256;
  const size_t off_tiles = off_reduce + (sizeof(ReduceItem) * n_items + 255) / 256 * 256;
  const size_t off_counter = off_tiles + (sizeof(BatchTile) * tiles.size() + 255) / 256 * 256;
  const size_t off_queue = off_counter + 256;
  const size_t total = off_queue + (sizeof(TileQueue) + 255) / 256 * 256;
  hipError_t e = hipMalloc(&p->mem, total);
  if (e != hipSuccess) {
    delete p;
    return fail(TDX_ERR_ALLOC, "plan allocation of %zu bytes failed", total);
  }
  char *base = (char *)p->mem;
  for (int i = 0; i < n_items; ++i) {
    bi[i].part = (double2 *)(base + part_off[i]);
    bi[i].tpart = bi[i].part + (size_t)bi[i].n_w * bi[i].n_g * bi[i].n_g *
                                   ri[i].n_slices;
    ri[i].part = bi[i].part;
    ri[i].tpart = bi[i].tpart;
  }
  p->items = (BatchItem *)(base + off_items);
  p->reduce = (ReduceItem *)(base + off_reduce);
  p->tiles = (BatchTile *)(base + off_tiles);
  p->counter = (int *)(base + off_counter);
  p->queue = (TileQueue *)(base + off_queue);
  p->n_tiles = (int)tiles.size();
  p->n_blocks = std::max(8, bf16x3_variant_occupancy(v) * std::max(ctx->n_cu, 1)) / 8 * 8;  // a multiple of the XCD count
  int rc = TDX_OK;
  const TileQueue q{p->items, p->tiles, p->n_tiles, p->counter};
  if (hipMemset(p->counter, 0, 256) != hipSuccess ||
      hipMemcpy(p->queue, &q, sizeof q, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->items, bi.data(), sizeof(BatchItem) * n_items, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(p->reduce, ri.data(), sizeof(ReduceItem) * n_items, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(p->tiles, tiles.data(), sizeof(BatchTile) * tiles.size(),
                hipMemcpyHostToDevice) != hipSuccess)
    rc = fail(TDX_ERR_HIP, "plan upload failed");
  if (rc != TDX_OK) {
    hipFree(p->mem);
    delete p;
    return rc;
  }
  *out = p;
  return TDX_OK;
}

int tdx_chi0_plan_launch(tdx_ctx *ctx, tdx_chi0_plan *p, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && p, TDX_ERR_INVALID_ARG, "null argument");
  hipStream_t s = as_stream(stream);
  if (p->prec != TDX_PREC_BF16X3) {
    for (const tdx_chi0_item &it : p->host_items)
      TDX_TRY(tdx_chi0(ctx, it.tl, it.n_trans, it.P, it.n_g, p->prec, it.omega, it.n_w, it.eta,
                       it.pref, it.chi0, stream));
    return TDX_OK;
  }
  TDX_TRY(bf16x3_launch_persistent(p->variant, p->queue, p->n_blocks, s));
  const unsigned rb = (unsigned)std::min<size_t>((p->max_per_slice + 255) / 256, 4096);
  hipLaunchKernelGGL(k_reduce_batch, dim3(rb, p->n_items), dim3(256), 0, s, p->reduce);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

int tdx_chi0_plan_destroy(tdx_chi0_plan *p) {
  clear_error();
  if (!p) return TDX_OK;
  if (p->mem) {
    hipSetDevice(p->device);
    hipDeviceSynchronize();
    hipFree(p->mem);
  }
  delete p;
  return TDX_OK;
}

int tdx_chi0_batched(tdx_ctx *ctx, const tdx_chi0_item *items, int n_items, int prec,
                     tdx_stream stream) {
  tdx_chi0_plan *p = nullptr;
  TDX_TRY(tdx_chi0_plan_create(ctx, items, n_items, prec, &p));
  int rc = tdx_chi0_plan_launch(ctx, p, stream);
  if (rc == TDX_OK && hipStreamSynchronize(as_stream(stream)) != hipSuccess)
    rc = fail(TDX_ERR_HIP, "stream synchronisation failed");
  tdx_chi0_plan_destroy(p);
  return rc;
}

int tdx_autotune_chi0(tdx_ctx *ctx, const tdx_chi0_item *probe, int prec, int64_t max_trans,
                      int *best_variant, int *best_slice_log2, double *best_ms) {
  clear_error();
  TDX_REQUIRE(ctx && probe && best_variant && best_slice_log2 && best_ms, TDX_ERR_INVALID_ARG,
              "null argument");
  TDX_REQUIRE(prec >= TDX_PREC_FP64 && prec <= TDX_PREC_BF16X3, TDX_ERR_INVALID_ARG, "bad prec");
  TDX_REQUIRE(probe->tl && probe->P && probe->omega && probe->chi0, TDX_ERR_INVALID_ARG,
              "probe has a null pointer");
  TDX_TRY(check_device(ctx));
  const long long nt = std::min<long long>(probe->n_trans, std::max<int64_t>(max_trans, 1));
  const int ld = (probe->n_g + 15) / 16 * 16;
  hipStream_t s = nullptr;
  TDX_HIP(hipStreamCreate(&s));
  hipEvent_t e0, e1;
  TDX_HIP(hipEventCreate(&e0));
  TDX_HIP(hipEventCreate(&e1));
  const int slice_opts[] = {18, 20};
  double best = 1e300;
  int bv = 0, bs = 18;
  int rc = TDX_OK;
  // both launch forms of the probe: one grid launch, and a one-item plan
  // (persistent kernel) built for the variant under test
  const long long p_rows = probe->p_rows > 0 ? probe->p_rows : probe->n_trans;
  TDX_REQUIRE(probe->n_trans <= p_rows, TDX_ERR_SHAPE, "probe has n_trans above p_rows");
  tdx_chi0_item one = *probe;
  one.n_trans = nt;
  one.p_rows = p_rows;
  tdx_chi0_tune &slot = ctx->tune[prec][bucket_of(ld)];
  const tdx_chi0_tune saved = slot;
  auto timed = [&](auto &&enqueue) {
    double ms_best = 1e300;
    for (int rep = 0; rep < 3 && rc == TDX_OK; ++rep) {
      hipEventRecord(e0, s);
      rc = enqueue();
      hipEventRecord(e1, s);
      hipEventSynchronize(e1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) ms_best = std::min(ms_best, (double)ms);
    }
    return ms_best;
  };
  // FP32 / FP64: one grid launch per variant (their slices fill the chip;
  // there is no persistent form)
  for (int v = 0; prec != TDX_PREC_BF16X3 && v < variant_count(prec) && rc == TDX_OK; ++v) {
    slot.variant = v;
    const double ms_best = timed([&] {
      return tdx_chi0(ctx, probe->tl, nt, probe->P, probe->n_g, prec, probe->omega, probe->n_w,
                      probe->eta, probe->pref, probe->chi0, (tdx_stream)s);
    });
    slot = saved;
    if (rc == TDX_OK && ms_best < best) {
      best = ms_best;
      bv = v;
      bs = saved.slice_log2;
    }
  }
  for (int v = 0; prec == TDX_PREC_BF16X3 && v < bf16x3_variant_count() && rc == TDX_OK; ++v) {
    for (int sl : slice_opts) {
      double ms_best = timed([&] {
        return chi0_bf16x3_with(ctx, v, sl, probe->P, p_rows, ld, probe->tl->delta,
                                probe->tl->df, (int)probe->tl->paired, nt, probe->omega,
                                probe->n_w, probe->eta, probe->n_g, probe->pref,
                                (double2 *)probe->chi0, s);
      });
      if (rc != TDX_OK) break;
      slot.variant = v;
      slot.slice_log2 = sl;
      tdx_chi0_plan *pl = nullptr;
      rc = tdx_chi0_plan_create(ctx, &one, 1, TDX_PREC_BF16X3, &pl);
      if (rc == TDX_OK) ms_best += timed([&] { return tdx_chi0_plan_launch(ctx, pl, s); });
      if (pl) tdx_chi0_plan_destroy(pl);
      slot = saved;
      if (rc != TDX_OK) break;
      if (ms_best < best) {
        best = ms_best;
        bv = v;
        bs = sl;
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipStreamDestroy(s);
  if (rc != TDX_OK) return rc;
  tdx_chi0_tune &t = ctx->tune[prec][bucket_of(ld)];
  t.variant = bv;
  t.slice_log2 = bs;
  t.ms = best;
  *best_variant = bv;
  *best_slice_log2 = bs;
  *best_ms = best;
  return TDX_OK;
}

int tdx_tune_save(tdx_ctx *ctx, const char *path) {
  clear_error();
  TDX_REQUIRE(ctx && path, TDX_ERR_INVALID_ARG, "null argument");
  FILE *f = std::fopen(path, "w");
  TDX_REQUIRE(f, TDX_ERR_INVALID_ARG, "cannot write %s", path);
  std::fprintf(f, "{\"arch\": \"gfx950\", \"entries\": [\n");
  bool first = true;
  for (int p = TDX_PREC_FP64; p <= TDX_PREC_BF16X3; ++p)
    for (int b = 0; b < 64; ++b) {
      const tdx_chi0_tune &t = ctx->tune[p][b];
      if (t.variant < 0) continue;
      std::fprintf(f,
                   "%s  {\"prec\": \"%s\", \"blocks\": %d, \"variant\": %d, \"slice_log2\": %d, "
                   "\"ms\": %.4f}",
                   first ? "" : ",\n", prec_name(p), b, t.variant, t.slice_log2, t.ms);
      first = false;
    }
  std::fprintf(f, "\n]}\n");
  std::fclose(f);
  return TDX_OK;
}

int tdx_tune_load(tdx_ctx *ctx, const char *path) {
  clear_error();
  TDX_REQUIRE(ctx && path, TDX_ERR_INVALID_ARG, "null argument");
  FILE *f = std::fopen(path, "r");
  TDX_REQUIRE(f, TDX_ERR_INVALID_ARG, "cannot read %s", path);
  char line[512];
  bool arch_ok = false;
  int loaded = 0;
  while (std::fgets(line, sizeof(line), f)) {
    if (std::strstr(line, "\"arch\": \"gfx950\"")) arch_ok = true;
    int b, v, sl;
    double ms;
    char pn[16] = "bf16x3";
    // entries name their precision; entries without one (older caches)
    // are split-BF16
    const bool with_prec =
        std::sscanf(line, " {\"prec\": \"%15[a-z0-9]\", \"blocks\": %d, \"variant\": %d, "
                          "\"slice_log2\": %d, \"ms\": %lf}", pn, &b, &v, &sl, &ms) == 5;
    if (arch_ok && (with_prec || std::sscanf(line, " {\"blocks\": %d, \"variant\": %d, "
                                                  "\"slice_log2\": %d, \"ms\": %lf}",
                                             &b, &v, &sl, &ms) == 4)) {
      int p = -1;
      for (int q = TDX_PREC_FP64; q <= TDX_PREC_BF16X3; ++q)
        if (std::strcmp(pn, prec_name(q)) == 0) p = q;
      if (p >= 0 && b >= 0 && b < 64 && v >= 0 && v < variant_count(p) && sl >= 10 && sl <= 30) {
        ctx->tune[p][b] = tdx_chi0_tune{v, sl, ms};
        ++loaded;
      }
    }
  }
  std::fclose(f);
  TDX_REQUIRE(arch_ok, TDX_ERR_UNSUPPORTED, "%s is not a gfx950 tuning cache", path);
  return TDX_OK;
}

}  // extern "C"
