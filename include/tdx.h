/*
 * tdx.h -- C ABI of the MI355X (gfx950) library for the linear-response
 * TDDFT route to the dynamic structure factor and the imaginary-time
 * correlation function of arXiv 2510.01875:
 *
 *   Kohn-Sham states -> transitions -> pair densities -> chi0 (Adler-Wiser)
 *   -> Dyson with K = v + f_xc -> S(q,w) (Eq. 8, detailed balance)
 *   -> F(q,tau) (Eq. 1).
 *
 * Units: Hartree atomic units throughout.
 *
 * Conventions shared by every entry point
 *  - Return value: TDX_OK (0) or a negative TDX_ERR_* code.  On error the
 *    outputs are left unchanged unless stated otherwise and tdx_last_error()
 *    returns a message for the calling thread.  Nothing throws or aborts
 *    across this boundary.
 *  - "device" pointers are HIP device allocations owned by the caller; the
 *    library never frees them.  "host" pointers are read (or written)
 *    before the call returns.  Workspaces are owned by the context.
 *  - Work is enqueued on the given HIP stream (NULL = default stream) in a
 *    fixed order; results are bitwise reproducible run to run.  Calls that
 *    must read a count or a status back to the host synchronise the stream;
 *    their descriptions say so.
 *  - Arrays are row-major.  Complex numbers are stored as interleaved
 *    (re, im) pairs of the stated real type.
 *  - Miller triples m give G = m1 b1 + m2 b2 + m3 b3 (b_i reciprocal rows).
 *  - k-points form the Monkhorst-Pack grid
 *      k_r = sum_i (2 r_i + 1 - N_i) / (2 N_i) b_i,  r_i = 0..N_i-1,
 *    flattened with r_3 fastest.  A momentum transfer is given by an integer
 *    triple qj: q = sum_i qj_i / N_i b_i, so that k + q = k' + G_s exactly.
 */
#ifndef TDX_H
#define TDX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TDX_ABI_VERSION 2

enum {
  TDX_OK = 0,
  TDX_ERR_INVALID_ARG = -1, /* null pointer, bad enum, non-finite input   */
  TDX_ERR_SHAPE = -2,       /* sizes inconsistent or capacity too small    */
  TDX_ERR_ALLOC = -3,       /* workspace above the context limit / OOM     */
  TDX_ERR_HIP = -4,         /* a HIP / rocSOLVER call failed               */
  TDX_ERR_NUMERIC = -5,     /* singular Dyson matrix, NaN, no mu bracket   */
  TDX_ERR_UNSUPPORTED = -6  /* device is not gfx950                        */
};

/* Arithmetic of the chi0 contraction.  Weights, states, Dyson and S/F are
 * always FP64. */
enum {
  TDX_PREC_FP64 = 0,   /* FP64 products, FP64 accumulation (MFMA f64)     */
  TDX_PREC_FP32 = 1,   /* FP32 products, FP32 accumulation per K-chunk,   */
                       /* FP64 across chunks                               */
  TDX_PREC_BF16X3 = 2  /* x = hi + lo (bf16, round-to-nearest-even),       */
                       /* hi*hi + hi*lo + lo*hi in FP32 per K-chunk, FP64  */
                       /* across chunks                                    */
};

enum { TDX_XC_RPA = 0, TDX_XC_ALDA = 1 };

typedef struct tdx_ctx tdx_ctx;
typedef void *tdx_stream; /* hipStream_t */

/* ------------------------------------------------------------------ */
/* Context                                                              */
/* ------------------------------------------------------------------ */

/* Create a context on HIP device `device`.  Fails with UNSUPPORTED if the
 * device is not gfx950.  *out receives the context (host). */
int tdx_create(int device, tdx_ctx **out);
int tdx_destroy(tdx_ctx *ctx);
/* Message of the last failed call on this thread ("" if none). */
const char *tdx_last_error(void);
int tdx_abi_version(void);
/* Cap on the library-owned workspace (bytes, 0 = no cap).  A call whose
 * workspace would exceed the cap fails with TDX_ERR_ALLOC before it writes
 * any output. */
int tdx_set_workspace_limit(tdx_ctx *ctx, size_t bytes);

/* ------------------------------------------------------------------ */
/* Model and Kohn-Sham states (FP64)                                   */
/* ------------------------------------------------------------------ */

/* Local pseudopotential V(G) = v(|G|) sum_I exp(-i G.R_I), V(0) = 0.
 * v on the shells |G|^2 = shell_unit^2 * shell_n2[j] is shell_v[j]; off
 * those shells v = 0, or, if gauss != 0, the Gaussian-regularised Coulomb
 * form factor -4 pi Z exp(-sigma^2 G^2/2) / (Omega G^2).  The model is
 * non-self-consistent (the paper's states are self-consistent DFT,
 * Sec. A.1). */
typedef struct {
  double cell[9];          /* rows a1, a2, a3 (bohr)                       */
  int kgrid[3];            /* Monkhorst-Pack sizes                         */
  double ecut_wf;          /* plane waves with 1/2|k+G|^2 <= ecut_wf       */
  int n_bands;             /* bands kept, moved up to the end of a         */
                           /* multiplet (gap < 1e-6 Ha); 0 = all           */
  double n_electrons;      /* electrons per cell (spin-unpolarised)        */
  double f_trunc;          /* the highest kept band must have f < f_trunc  */
  int n_atoms;             /* ions                                         */
  const double *positions; /* host [n_atoms][3] cartesian bohr             */
  double shell_unit;       /* bohr^-1                                      */
  int n_shells;
  const int *shell_n2;     /* host [n_shells]                              */
  const double *shell_v;   /* host [n_shells] Ha                           */
  int gauss;               /* 0/1                                          */
  double z_ion, sigma;
} tdx_model;

typedef struct {
  int n_k;      /* prod(kgrid)                                             */
  int npw_max;  /* largest plane-wave basis over the grid                  */
  int nb_max;   /* band capacity: n_bands + 64 (or npw_max if all)         */
} tdx_states_dims;

/* Host-only: sizes needed by tdx_build_states. */
int tdx_states_query(const tdx_model *model, tdx_states_dims *out);

/* Device-resident states.  The caller allocates every buffer with the
 * sizes from tdx_states_query and fills in the pointers and dims. */
typedef struct {
  int n_k, npw_max, nb_max;
  int *npw;       /* device [n_k]                                          */
  int *nb;        /* device [n_k] kept band count                          */
  int *miller;    /* device [n_k][npw_max][3], basis of each k             */
  double *eps;    /* device [n_k][nb_max] eigenvalues, ascending           */
  double *occ;    /* device [n_k][nb_max] Fermi-Dirac occupations          */
  double *coef;   /* device complex128 [n_k][nb_max][npw_max], band rows,  */
                  /* zero beyond npw[k]                                    */
  int kgrid[3];       /* out (host): Monkhorst-Pack sizes                  */
  int mmax[3];        /* out (host): largest |Miller index| per axis       */
  double cell[9];     /* out (host): rows a1, a2, a3                       */
  double bvec[9];     /* out (host): reciprocal rows b1, b2, b3            */
  double mu;          /* out (host): chemical potential                    */
  double temperature; /* out (host)                                        */
  double omega_cell;  /* out (host): cell volume                           */
  double n_electrons; /* out (host): electrons per cell of the occupations */
  double beta;        /* out (host): 1 / temperature                       */
  double density;     /* out (host): n = n_electrons / omega_cell, the     */
                      /* electron density of the FDT (tdx_dsf)             */
  double chi0_pref;   /* out (host): 2 / (n_k omega_cell), the Adler-Wiser */
                      /* normalisation (spin-unpolarised) of tdx_chi0      */
} tdx_states;

/* Plane-wave Hamiltonian H_GG'(k) = 1/2|k+G|^2 delta + V(G-G') on every
 * k of the grid, dense FP64 eigensolve, band count snapped to a multiplet
 * end, chemical potential by bisection on (2/N_k) sum f = N_e, Fermi-Dirac
 * occupations at `temperature`.  Writes every "out (host)" field of st,
 * among them the density and the chi0 normalisation that tdx_dsf and
 * tdx_chi0 take.  Synchronises the stream.
 * Errors: SHAPE if the snapped band count exceeds nb_max, NUMERIC if the
 * top kept band has f >= f_trunc or the electron count cannot be met. */
int tdx_build_states(tdx_ctx *ctx, const tdx_model *model, double temperature,
                     tdx_states *st, tdx_stream stream);

/* Occupations and mu of existing states at another temperature (same
 * orbitals: the model is non-self-consistent); updates mu, temperature,
 * beta, n_electrons, density and chi0_pref of st.  Synchronises. */
int tdx_occupations(tdx_ctx *ctx, tdx_states *st, double temperature,
                    double n_electrons, double f_trunc, tdx_stream stream);

/* ------------------------------------------------------------------ */
/* Response basis (host geometry)                                      */
/* ------------------------------------------------------------------ */

/* B(q) = {G : 1/2|q+G|^2 <= ecut_chi, q+G != 0}, sorted by |q+G|^2 then
 * Miller triple.  Writes up to `capacity` triples to miller_out (host,
 * [capacity][3]), the count to *n_out and the index of G = 0 (the
 * reported q+G = q element) to *i_g0.  SHAPE if capacity is too small
 * (*n_out still set); INVALID_ARG if G = 0 is outside the basis. */
int tdx_response_basis(const double cell[9], const int kgrid[3], const int qj[3],
                       double ecut_chi, int *miller_out, int capacity, int *n_out,
                       int *i_g0);

/* Host-only: the momentum transfer q = sum_i (qj_i / kgrid_i) b_i in
 * Cartesian coordinates (q_out host [3], may be null) and |q|^2 (q2_out,
 * may be null), the |q + G|^2 of the reported element G = 0 that the
 * dielectric step (tdx_dielectric) takes. */
int tdx_momentum(const double cell[9], const int kgrid[3], const int qj[3], double *q_out,
                 double *q2_out);

/* ------------------------------------------------------------------ */
/* Transitions                                                          */
/* ------------------------------------------------------------------ */

/* T(q) = {(k,n,m): |f_nk - f_m,k+q| > thr}, ordered by k, then n, then m.
 * Device arrays of capacity `capacity` entries (caller-owned):
 *   k[T] int32, n[T] int32, m[T] int32,
 *   delta[T] = eps_m(k+q) - eps_n(k) (FP64), df[T] = f_n - f_m (FP64),
 *   k_offsets[n_k + 1] int64 (CSR by k).
 * The count is always written to *count (host).  With capacity < count
 * nothing else is written and SHAPE is returned: call once with
 * capacity 0 to size the buffers.  A call whose pointers are all null is
 * such a count query and returns OK when the set is empty.  Otherwise
 * k_offsets must be given, and the five per-transition arrays too unless
 * the set is empty (INVALID_ARG).  Synchronises.
 *
 * paired (input, 0 or 1): with 1 the list keeps one transition of each
 * time-reversal pair.  For a real local potential without spin-orbit
 * coupling on an inversion-symmetric k-grid, the transition
 * (k, n -> k+q, m) and its partner (-k-q, m -> -k, n) have the same rho rho^H
 * (summed over degenerate multiplets), opposite delta and opposite df, so
 * the two Adler-Wiser terms combine into one with the weight
 *   df [1/(w - delta + i eta) - 1/(w + delta + i eta)]
 *     = 2 df delta / ((w + i eta)^2 - delta^2).
 * The kept k are those whose partner index (-k-q on the grid) is larger;
 * a k that is its own partner keeps n < m.  tdx_chi0 and the batch plans
 * then apply the combined weight (chi0 equals that of the full list up to
 * rounding); pair densities are computed for the kept transitions only.
 * The reverse-mode entry points differentiate the combined weight; they
 * attribute each pair's cotangents to the states of its kept transition,
 * which, by the same symmetry, leaves the gradients in T, eta and the
 * potential those of the full list. */
typedef struct {
  int64_t capacity;
  int *k, *n, *m;
  double *delta, *df;
  int64_t *k_offsets;
  int32_t paired;
} tdx_translist;

int tdx_transitions(tdx_ctx *ctx, const tdx_states *st, const int qj[3],
                    double thr, tdx_translist *tl, int64_t *count,
                    tdx_stream stream);

/* ------------------------------------------------------------------ */
/* Pair densities                                                       */
/* ------------------------------------------------------------------ */

/* rho_t(G) = <n k| e^{-i(q+G).r} |m k+q> = sum_G1 c*_nk(G1) c_m,k'(G1+G+G_s)
 * for the first n_trans transitions of the list and every response vector G
 * (basis from tdx_response_basis, copied to device: gbasis [n_g][3] int32).
 * Computed in FP64 (MFMA); stored per `prec` with row stride ld = n_g rounded
 * up to a multiple of 16 (zero-padded):
 *   FP64:   complex128 P[T][ld]
 *   FP32:   complex64  P[T][ld]
 *   BF16X3: with x32 = fp32(x), hi = RNE_bf16(x32), lo = RNE_bf16(x32 - hi)
 *           and T' = T rounded up to 32 plus 32 (rows past T are zero):
 *           fragment words uint32 [T'/4][2][ld][4]: for each quad of
 *           transitions and column, the two 16-byte groups hi and lo, each
 *           word a (re, im) bf16 pair (re in the low half), the last index
 *           the transition in the quad; then complex64 x32 rows [T'][ld]
 *           (16 bytes per row and column in all).
 * P must hold tdx_pair_density_bytes(...) bytes.  tdx_chi0 must be given the
 * same n_trans as the buffer was written for (the split-BF16 layout depends
 * on it). */
size_t tdx_pair_density_bytes(int64_t n_trans, int n_g, int prec);
int tdx_pair_density(tdx_ctx *ctx, const tdx_states *st, const int qj[3],
                     const tdx_translist *tl, int64_t n_trans,
                     const int *gbasis, int n_g, int prec, void *P,
                     tdx_stream stream);
/* The same for the transitions t_begin .. t_end - 1 of the list, stored as
 * rows 0 .. t_end - t_begin - 1 of P (the layout above for t_end - t_begin
 * transitions): a list can be processed in blocks whose buffers are
 * recomputed rather than held (the reverse sweep does this).  Equal, row for
 * row, to the rows of a whole-list call. */
int tdx_pair_density_range(tdx_ctx *ctx, const tdx_states *st, const int qj[3],
                           const tdx_translist *tl, int64_t t_begin, int64_t t_end,
                           const int *gbasis, int n_g, int prec, void *P, tdx_stream stream);
/* tdx_pair_density_range without allocation, host copy, memset or
 * synchronisation (graph-capturable): its tables (Miller lookups, row and
 * column groups, k + q maps) are built by kernels in `work`, a caller-owned
 * device buffer of at least tdx_pair_density_work_bytes(st, t_end - t_begin)
 * bytes (SHAPE otherwise) that must stay alive until the stream has run the
 * call.  Same results as tdx_pair_density_range. */
size_t tdx_pair_density_work_bytes(const tdx_states *st, int64_t n_trans);
int tdx_pair_density_async(tdx_ctx *ctx, const tdx_states *st, const int qj[3],
                           const tdx_translist *tl, int64_t t_begin, int64_t t_end,
                           const int *gbasis, int n_g, int prec, void *P, void *work,
                           size_t work_bytes, tdx_stream stream);

/* ------------------------------------------------------------------ */
/* chi0 (Adler-Wiser), the MFMA contraction                             */
/* ------------------------------------------------------------------ */

/* chi0_GG'(q,w) = pref * sum_t df_t / (w - delta_t + i eta) rho_t(G) rho_t(G')*
 * with pref the normalisation 2 / (N_k Omega) of the states (their
 * chi0_pref field; another value scales the result).  The weights are
 * formed in FP64 in-kernel; the products run in `prec` (see TDX_PREC_*).
 * omega: device [n_w] FP64.  chi0: device complex128 [n_w][n_g][n_g].
 * The sum over t is split into fixed chunks reduced in a fixed order, so a
 * call is bitwise reproducible on one device; the split-BF16 slice count
 * depends on the list's shape and the device's CU count
 * (tdx_chi0_bf16x3_slicing), and a length fixed with
 * tdx_chi0_set_slice_length makes the rounding order the same on every
 * device. */
int tdx_chi0(tdx_ctx *ctx, const tdx_translist *tl, int64_t n_trans,
             const void *P, int n_g, int prec, const double *omega, int n_w,
             double eta, double pref, double *chi0, tdx_stream stream);

/* ------------------------------------------------------------------ */
/* Ragged batches of q in one persistent launch, tile autotuning        */
/* ------------------------------------------------------------------ */

/* One q-vector of a batch (all pointers device, as for tdx_chi0). */
typedef struct {
  const tdx_translist *tl; /* host struct; its arrays are device            */
  int64_t n_trans;
  const void *P;           /* pair densities of this q in the plan's prec   */
  int n_g;
  const double *omega;     /* device [n_w]                                  */
  int n_w;
  double eta, pref;
  double *chi0;            /* device complex128 [n_w][n_g][n_g], output     */
  int64_t p_rows;          /* transitions P was written for (0: n_trans);   */
                           /* the first n_trans <= p_rows are contracted    */
} tdx_chi0_item;

typedef struct tdx_chi0_plan tdx_chi0_plan;

/* Build the work queue of a ragged batch: for TDX_PREC_BF16X3 every
 * (q, frequency block, G block, G' block, transition slice) tile, ordered
 * by predicted cost, costliest first, plus the slice-partial buffers and the
 * queue counter, in one device allocation owned by the plan.  Every item is
 * sliced as a grid launch of it would be, so the plan's results are bitwise
 * those of one tdx_chi0 call per item (same configuration).  The tile shape is the configured one (see
 * tdx_chi0_set_config / tdx_autotune_chi0) of the widest basis in the batch.
 * Other precisions run their items one launch each.  Items must stay valid
 * until the plan is destroyed. */
int tdx_chi0_plan_create(tdx_ctx *ctx, const tdx_chi0_item *items, int n_items, int prec,
                         tdx_chi0_plan **out);
/* Enqueue the plan: ONE persistent kernel (the variant's workgroups per CU
 * on every CU) whose workgroups take tiles off the list one at a time
 * through the plan's atomic counter, which the kernel sets back to zero as it
 * ends, and one batched slice reduction.  No allocation, host
 * synchronisation or memset: the launch can be captured into a HIP graph and
 * replayed.  Results are independent of which workgroup ran which tile
 * (fixed-order FP64 slice reduction).  Launches of one plan must not overlap
 * (they share its partials and counter). */
int tdx_chi0_plan_launch(tdx_ctx *ctx, tdx_chi0_plan *plan, tdx_stream stream);
int tdx_chi0_plan_destroy(tdx_chi0_plan *plan);
/* create + launch + synchronise + destroy */
int tdx_chi0_batched(tdx_ctx *ctx, const tdx_chi0_item *items, int n_items, int prec,
                     tdx_stream stream);

/* Number of tile variants of a precision (frequencies per wave x G' per
 * workgroup x chunk, and for split-BF16 buffering and waves per workgroup). */
int tdx_chi0_variants(int prec, int *count);
/* Tile variant (-1 = default: for split-BF16 the 8-wave 2 x 9 tile with three
 * LDS buffers, for FP32 and FP64 variant 0) and slice length 2^slice_log2
 * (default 2^20; split-BF16 only, the FP32 and FP64 kernels choose their
 * slices to fill the chip) used for bases of n_g vectors (size classes of
 * 16), per precision. */
int tdx_chi0_set_config(tdx_ctx *ctx, int prec, int n_g, int variant, int slice_log2);
int tdx_chi0_get_config(tdx_ctx *ctx, int prec, int n_g, int *variant, int *slice_log2);
/* Slice length of every later chi0 contraction on this context (all
 * precisions, grid launches and plans): with n > 0 the transition list of a
 * q is cut into slices of n transitions (rounded up to the kernel's chunk),
 * the last one shorter, whatever the tile count; n = 0 (the default) lets
 * each call choose the length (the tuned 2^slice_log2, shortened until the
 * tiles fill the chip; then, for split-BF16, the slice count up to 4 times
 * that whose rounds of tiles leave the least predicted idle time).  Within a slice the sums run in FP32 over runs of
 * chunks (split-BF16, FP32) and in FP64 across runs; the slices' FP64
 * partials are reduced in a fixed order, so the length fixes the rounding
 * order and the partial workspace (slices x n_w x n_g^2 x 16 bytes). */
int tdx_chi0_set_slice_length(tdx_ctx *ctx, int64_t n);
/* The slicing a split-BF16 contraction takes with no fixed length set (host
 * only, no device or context needed): for a list of n_trans transitions, a
 * basis of n_g vectors, n_w frequencies, tile variant `variant`
 * (0 .. tdx_chi0_variants - 1), minimum slice length 2^slice_log2 and n_cu
 * compute units, the slice length (*slice_len, a multiple of the 32-transition
 * chunk) and count (*slices) whose rounds of tiles leave the least predicted
 * idle time; the count lies between the minimum (2^slice_log2 transitions a
 * slice, at least 2048 tiles) and 4 times it.  TDX_ERR_INVALID_ARG for null
 * outputs or sizes out of range. */
int tdx_chi0_bf16x3_slicing(int n_cu, int variant, int64_t n_trans, int n_g, int n_w,
                            int slice_log2, int64_t *slice_len, int *slices);

/* Time every variant of `prec` on the probe item (its first max_trans
 * transitions, P in that precision's layout; probe->chi0 is overwritten),
 * keep the fastest for the probe's size class in the context and return it.
 * Split-BF16: every variant and slice length 2^{18,20} in both launch forms,
 * one grid launch and a one-item plan (the persistent kernel), ranked by the
 * sum of the two times (best_ms); FP32 and FP64: one grid launch per variant
 * (best_slice_log2 returns the unused stored value).  Allocates; synchronises. */
int tdx_autotune_chi0(tdx_ctx *ctx, const tdx_chi0_item *probe, int prec, int64_t max_trans,
                      int *best_variant, int *best_slice_log2, double *best_ms);
/* Tuning cache as JSON text keyed by the gfx arch, one entry per precision
 * and size class. */
int tdx_tune_save(tdx_ctx *ctx, const char *path);
int tdx_tune_load(tdx_ctx *ctx, const char *path);

/* ------------------------------------------------------------------ */
/* Kernel K = v + f_xc and the Dyson solve (FP64)                      */
/* ------------------------------------------------------------------ */

/* K_GG' = 4 pi / |q+G|^2 delta_GG' + f_xc(G - G').  For TDX_XC_ALDA,
 * f_xc(G) = (1/N_r) sum_j f_xc(n(r_j)) e^{-i G.r_j} on the real-space
 * grid r_j = sum_i (j_i/N_i) a_i (dens_grid[3]), with
 * n(r_j) = 2/(N_k Omega) sum_kn f_nk |sum_G c_nk(G) e^{i G.r_j}|^2 and
 * f_xc = d^2(n eps_xc)/dn^2 for Slater exchange + PW92 correlation (the
 * local form of the paper's adiabatic kernel, Sec. A.1).  States with
 * f_nk < 1e-20 are skipped (their weight is below FP64 resolution).
 * K: device complex128 [n_g][n_g].  SHAPE if a grid side is smaller than
 * the span of a wavefunction basis.  Synchronises for ALDA.  Equal to
 * tdx_xc_kernel_grid followed by tdx_kernel_matrix_from_grid. */
int tdx_kernel_matrix(tdx_ctx *ctx, const tdx_states *st, const int qj[3],
                      const int *gbasis, int n_g, int xc, const int dens_grid[3],
                      double *K, tdx_stream stream);

/* The q-independent part of the ALDA kernel: f_xc(G) on the full FFT grid
 * of dens_grid[3] (as defined above), for the states' current occupations.
 * fxg: device complex128 [N0][N1][N2], caller-owned, index
 * ((G_0 mod N0) N1 + (G_1 mod N1)) N2 + (G_2 mod N2).  A grid stays valid
 * until the occupations change (tdx_occupations).  Same SHAPE errors as
 * tdx_kernel_matrix; synchronises. */
int tdx_xc_kernel_grid(tdx_ctx *ctx, const tdx_states *st, const int dens_grid[3], double *fxg,
                       tdx_stream stream);

/* K for one q from a grid of tdx_xc_kernel_grid (ignored for TDX_XC_RPA,
 * where fxg may be null).  Bitwise equal to tdx_kernel_matrix on the same
 * states.  Asynchronous; fxg must stay alive until the stream reaches it. */
int tdx_kernel_matrix_from_grid(tdx_ctx *ctx, const tdx_states *st, const int qj[3],
                                const int *gbasis, int n_g, int xc, const int dens_grid[3],
                                const double *fxg, double *K, tdx_stream stream);

/* chi_{00}(w) for every w: solve (1 - chi0(w) K) x = chi0(w) e_{i_g0} by LU
 * with partial pivoting and return x_{i_g0}.  chi0: device complex128
 * [n_w][n_g][n_g]; K: device complex128 [n_g][n_g]; chi00 out: device
 * complex128 [n_w].  Synchronises to check pivots: NUMERIC if a pivot is
 * zero or not finite (outputs then undefined for that w only). */
int tdx_dyson(tdx_ctx *ctx, const double *chi0, const double *K, int n_g,
              int n_w, int i_g0, double *chi00, tdx_stream stream);

/* tdx_dyson for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same per-frequency LU solves and results as tdx_dyson (bitwise), with the
 * matrices 1 - chi0 K and the pivot status in a fixed library-owned device
 * array of tdx_dyson_noalloc_max_bytes() bytes (64 MiB; each GPU holds its
 * own copy until the process ends) instead of the context workspace.  The
 * frequencies run in passes of as many as the array holds.  Calls no
 * allocator; the caller passes chi0, K and chi00 as for tdx_dyson.
 * Synchronises the stream to read the pivot status: NUMERIC if a pivot is
 * zero or not finite (chi00 NaN for that frequency).  SHAPE if one matrix
 * (16 n_g^2 bytes) does not fit the array.  Every call on a GPU shares its
 * array: calls that overlap on one GPU (several streams or threads) race. */
size_t tdx_dyson_noalloc_max_bytes(void);
int tdx_dyson_noalloc(tdx_ctx *ctx, const double *chi0, const double *K, int n_g, int n_w,
                      int i_g0, double *chi00, tdx_stream stream);

/* tdx_dyson without allocation or synchronisation (graph-capturable):
 * work is a caller-owned device buffer of tdx_dyson_work_bytes(n_g, n_w)
 * bytes, info a device int [n_w] that receives 0 or the failing column + 1
 * (chi00 is NaN for that frequency). */
size_t tdx_dyson_work_bytes(int n_g, int n_w);
int tdx_dyson_async(tdx_ctx *ctx, const double *chi0, const double *K, int n_g, int n_w,
                    int i_g0, double *chi00, void *work, int *info, tdx_stream stream);

/* ------------------------------------------------------------------ */
/* S(q,w) and F(q,tau) (FP64)                                          */
/* ------------------------------------------------------------------ */

/* Fluctuation-dissipation theorem (Eq. 8) in the normalisation
 * S = -Im chi / (pi n (1 - e^{-beta w})), valid for either sign of w; at
 * w = 0 exactly S = -Im chi(w1) / (pi n beta w1) from the next point.
 * chi00: device complex128 [n_w]; omega, S: device FP64 [n_w]. */
int tdx_dsf(tdx_ctx *ctx, const double *chi00, const double *omega, int n_w,
            double beta, double density, double *S, tdx_stream stream);

/* Two-sided Laplace transform (Eq. 1) on the w >= 0 grid with the negative
 * half from detailed balance S(-w) = e^{-beta w} S(w):
 * F(tau) = sum_j c_j S_j (e^{-tau w_j} + e^{-(beta - tau) w_j}), c_j the
 * composite-trapezoid weights.  S, omega: device [n_w]; tau, F: device
 * [n_tau]. */
int tdx_itcf(tdx_ctx *ctx, const double *S, const double *omega, int n_w,
             double beta, const double *tau, int n_tau, double *F,
             tdx_stream stream);

/* ------------------------------------------------------------------ */
/* The eta-convergence test in imaginary time (Sec. 2, Eq. 2, Fig. 2)  */
/* ------------------------------------------------------------------ */

/* Metrics of n_set ITCFs F [n_set][n_tau] (device FP64) on one tau grid
 * (device [n_tau]) that starts at 0 and ends at beta or at beta/2 (then the
 * symmetry F(tau) = F(beta - tau) supplies the rest) and holds beta/2:
 * metrics (device FP64 [n_set][5]) = F(beta/2), A = int_0^beta F dtau,
 * F~(beta/2), int_0^beta F~ dtau = A - beta F(0), chi(q) = -n A, with the
 * shifted ITCF F~(tau) = F(tau) - F(0) of Eq. 2 and the integrals by the
 * composite trapezoid on the grid.  Asynchronous; a grid of another form
 * gives NaN metrics. */
int tdx_itcf_metrics(tdx_ctx *ctx, const double *F, int n_set, const double *tau, int n_tau,
                     double beta, double density, double *metrics, tdx_stream stream);

/* The reference eta of the test: eta (host [n_eta], increasing) and its
 * metrics (host [n_eta][5] from tdx_itcf_metrics); the convergence range is
 * the run of eta from the smallest one over which both shifted metrics,
 * F~(beta/2) and int_0^beta F~ dtau, stay within tol (relative) of their
 * values at the smallest eta, and *ref_index is the largest eta of that run
 * (the paper selects the largest converged eta by inspection; tol is this
 * library's reading of "converged").  NUMERIC if a metric is not finite. */
int tdx_eta_reference(const double *metrics, const double *eta, int n_eta, double tol,
                      int *ref_index);

/* ------------------------------------------------------------------ */
/* Dielectric properties from S (Sec. 3 and A.2, Eqs. 8, A-1, A-2)     */
/* ------------------------------------------------------------------ */

/* From S on an increasing grid 0 <= w_0 < ... (device [n_w]): Im chi by the
 * FDT in the normalisation of tdx_dsf, Im chi = -pi n (1 - e^{-beta w}) S;
 * Re chi by the Kramers-Kronig relation
 *   Re chi(w) = (2/pi) P int_0^{w_max} w' Im chi(w') / (w'^2 - w^2) dw'
 * with Im chi linear between grid points (closed form per interval; no tail
 * past the grid); eps^{-1} = 1 + (4 pi / q2) chi (Eq. A-1, q2 = |q + G|^2 of
 * the element); sigma = -i w (eps - 1) / (4 pi) (Eq. A-2).  Outputs are
 * device complex128 [n_w], each may be null.  Asynchronous; the grid is not
 * checked (one that does not increase gives non-finite values). */
int tdx_dielectric(tdx_ctx *ctx, const double *S, const double *omega, int n_w, double beta,
                   double density, double q2, double *chi, double *eps_inv, double *sigma,
                   tdx_stream stream);

/* ------------------------------------------------------------------ */
/* Attenuation of narrow-band fluctuations (Sec. 3, Eqs. 3-7, Figs. 3  */
/* and 4): S = S_p + S_n, S_p from a Savitzky-Golay filter whose       */
/* window and degree a scored grid search picks, subject to conditions */
/* on the residual F_n in imaginary time.  All FP64.  With a zero     */
/* filter, set or frequency count the outputs may be null and nothing  */
/* is written.                                                        */
/* ------------------------------------------------------------------ */

/* A bank of n_filt Savitzky-Golay filters applied to S (device [n_w],
 * samples taken as equally spaced): Sp[f][i] (device [n_filt][n_w]) is the
 * least-squares polynomial of degree degrees[f] over the windows[f] samples
 * centred on i, evaluated at i; near the ends the window is moved inside
 * the grid ([0, w) or [n_w - w, n_w)) and the same fit is evaluated at i.
 * hdiag (device [n_filt][n_w], may be null) receives the weight of S_i in
 * its own filtered value (the smoother's diagonal; its sum is the filter's
 * effective number of parameters).  windows, degrees: host [n_filt]; each
 * window odd, above its degree and at most n_w; degrees 0..8, else
 * INVALID_ARG.  Synchronises (the host lists are copied on the stream). */
int tdx_sg_filter(tdx_ctx *ctx, const double *S, int n_w, const int *windows,
                  const int *degrees, int n_filt, double *Sp, double *hdiag, tdx_stream stream);

/* Power spectrum of dS/dw, used to find the frequencies of the
 * fluctuations: with the central difference
 *   D_i = (S_{i+1} - S_{i-1}) / (w_{i+1} - w_{i-1}),  i = 1 .. n_w - 2,
 * psd[s][k] = |(1/(n_w - 2)) sum_i D_i exp(-2 pi i nu_k w_i)|^2, nu in
 * cycles per unit of w.  S: device [n_set][n_w], omega: device [n_w], nu:
 * device [n_nu], psd: device [n_set][n_nu].  Asynchronous. */
int tdx_derivative_psd(tdx_ctx *ctx, const double *S, const double *omega, int n_w, int n_set,
                       const double *nu, int n_nu, double *psd, tdx_stream stream);

/* Scores of each filter of a bank against the unfiltered S (all device):
 * scores[f] (device [n_filt][5]) = (RSS, k, AICc, P_freq, P_curv) with
 *   RSS = sum_i (Sp_i - S_i)^2,  k = sum_i hdiag_i,
 *   AICc = n ln(RSS / n) + 2k + 2k(k+1)/(n - k - 1)  (+inf if n - k - 1 <= 0),
 *   P_freq = mean over the n_nu target frequencies of the ratio of the
 *            power of dSp/dw to that of dS/dw (tdx_derivative_psd), 0 if
 *            n_nu = 0,
 *   P_curv = sum of squared second differences of Sp over those of S (NaN
 *            if S has none).
 * The two penalties are this library's reading of the paper's
 * frequency-domain and second-derivative penalties, whose forms it does not
 * give.  n_nu <= 16.  Asynchronous. */
int tdx_sg_scores(tdx_ctx *ctx, const double *S, const double *Sp, const double *hdiag,
                  const double *omega, int n_w, int n_filt, const double *nu, int n_nu,
                  double *scores, tdx_stream stream);

/* Imaginary-time conditions on the residual (Eqs. 5 and 7): for each set s,
 * F_n = F_ref - F_p[s] on the tau grid (device [n_tau], from 0 to beta or
 * to beta/2, holding beta/2, as for tdx_itcf_metrics) and
 *   out[s] = (max_tau |F_n / F_ref|,  Fbar_n / F_ref(beta/2),
 *             sigma_n / F_ref(beta/2)),
 *   Fbar_n = (1/beta) int_0^beta F_n dtau,
 *   sigma_n = ((1/beta) int_0^beta (F_n - Fbar_n)^2 dtau)^{1/2}
 * (Eq. 7 read as the root-mean-square deviation over [0, beta], so that the
 * ratios do not depend on the unit of tau), by the trapezoid rule; a grid
 * ending at beta/2 uses F_n(tau) = F_n(beta - tau).  F_ref: device [n_tau],
 * F_p: device [n_set][n_tau], out: device [n_set][3]; NaN for a grid of
 * another form.  Asynchronous. */
int tdx_residual_itcf(tdx_ctx *ctx, const double *F_ref, const double *F_p, int n_set,
                      const double *tau, int n_tau, double beta, double *out,
                      tdx_stream stream);

/* Selection of the grid search (host): the filter with the smallest
 *   J = AICc / n_w + lam_f P_freq + lam_c P_curv
 * over scores (host [n_filt][5] from tdx_sg_scores) among those whose
 * residual (host [n_filt][3] from tdx_residual_itcf, or null for none)
 * satisfies |Fbar_n / F_ref(beta/2)| <= mean_tol and
 * sigma_n / F_ref(beta/2) <= sigma_tol; filters with a non-finite J are
 * skipped.  *best = its index, or -1 if none qualifies.  The weights and
 * tolerances are the caller's (the paper gives neither); to pick the best
 * window per degree, call it on each degree's rows. */
int tdx_sg_select(const double *scores, const double *resid, int n_filt, int n_w, double lam_f,
                  double lam_c, double mean_tol, double sigma_tol, int *best);

/* ------------------------------------------------------------------ */
/* Kubo-Greenwood route (Sec. A.3, with Eqs. 8, A-1, A-2)               */
/* ------------------------------------------------------------------ */

/* The scaled structure factor S* = v(q) S of the optical limit from a
 * conductivity sigma (device complex128 [n_w], e.g. a Kubo-Greenwood
 * calculation's) on the grid omega (device [n_w], w >= 0):
 *   eps = 1 + 4 pi i sigma / w,  chi* = 1/eps - 1,
 *   S* = -Im chi* / (pi n (1 - e^{-beta w}))
 * (the normalisation of tdx_dsf; w = 0 takes the limit from the next grid
 * point, NaN without one).  S*: device [n_w].  F* (tdx_itcf), the eta
 * metrics, the attenuation and the way back run on S* unchanged; the way
 * back (Re chi* by Kramers-Kronig, eps^{-1} = 1 + chi*,
 * sigma = i w (1 - eps) / (4 pi)) is tdx_dielectric with q2 = 4 pi.
 * Asynchronous. */
int tdx_kg_dsf(tdx_ctx *ctx, const double *sigma, const double *omega, int n_w, double beta,
               double density, double *S_star, tdx_stream stream);

/* The Kubo-Greenwood conductivity of the states, the input of the route
 * above (Sec. A.3 starts from it; its eta test broadens it): the trace
 * average over the three Cartesian directions with every transition's
 * delta function broadened into a Lorentzian of half-width eta,
 *   sigma(w) = 2 i / (Omega N_k) sum_t W_t / (w - delta_t + i eta),
 *   W_t = (df_t / delta_t) (1/3) sum_a |<m k| p_a |n k>|^2,
 *   <m k| p_a |n k> = sum_G conj(c_mk(G)) (k + G)_a c_nk(G),  p = -i grad,
 * the factor 2 for the spins.  Re sigma is the usual
 * (2 pi / (3 Omega w)) sum (f_n - f_m) |p_mn|^2 delta(e_m - e_n - w) per
 * k-point weight 1/N_k, broadened; Im sigma is its Kramers-Kronig partner.
 * tl: the transitions of tdx_transitions at qj = (0, 0, 0) for these
 * states and occupations (delta = e_m - e_n, df = f_n - f_m; the screening
 * threshold of that call is the conductivity's), the full list (a paired
 * list is INVALID_ARG); n_trans its count (0 gives sigma = 0).  omega:
 * device [n_w]; sigma: device complex128 [n_w] (out).  work: device,
 * caller-owned, at least tdx_kg_work_bytes(n_trans, n_w) bytes (SHAPE if
 * smaller).  No allocation, memset or host synchronisation: a HIP graph
 * can hold the call. */
size_t tdx_kg_work_bytes(int64_t n_trans, int n_w);
int tdx_kg_conductivity(tdx_ctx *ctx, const tdx_states *st, const tdx_translist *tl,
                        int64_t n_trans, const double *omega, int n_w, double eta, double *sigma,
                        void *work, size_t work_bytes, tdx_stream stream);

/* ------------------------------------------------------------------ */
/* Reverse mode: vector-Jacobian products of F(q,tau) (FP64)           */
/* ------------------------------------------------------------------ */

/* Gradients of F(q,tau) (Eq. 1 with S from Eq. 8) with respect to the
 * temperature T, the broadening eta and the tabulated shell values v_s of
 * the potential, one call per step of the forward chain, run in reverse:
 *   itcf_vjp -> dsf_vjp -> dyson_vjp -> chi0_vjp -> weights_vjp
 *   -> occupations_vjp, pair_density_vjp (per q) -> potential_vjp (once).
 * A real cotangent xbar means dL = sum xbar dx; a complex one zbar means
 * dL = Re sum conj(zbar) dz.  The RPA kernel depends on none of T, eta,
 * v; the ALDA kernel's dependence through the density has three calls of
 * its own (after tdx_potential_vjp below).  Temperature enters through beta = 1/T in S and
 * F (the caller chains beta_bar and tau_bar) and through the occupations
 * (occupations_vjp).  Calls that accumulate ("+=") leave zeroing to the
 * caller so that several q can share one set of state cotangents. */

/* F(tau_j) = sum_i c_i S_i (e^{-tau_j w_i} + e^{-(beta - tau_j) w_i}).
 * F_bar: device [n_tau].  Writes S_bar [n_w], tau_bar [n_tau] and
 * beta_bar [1] (the explicit beta of the second exponential only). */
int tdx_itcf_vjp(tdx_ctx *ctx, const double *S, const double *omega, int n_w, double beta,
                 const double *tau, int n_tau, const double *F_bar, double *S_bar,
                 double *tau_bar, double *beta_bar, tdx_stream stream);

/* S = -Im chi00 / (pi n (1 - e^{-beta w})) (w = 0 from the next point).
 * Writes chi00_bar (device complex128 [n_w]) and beta_bar [1]. */
int tdx_dsf_vjp(tdx_ctx *ctx, const double *chi00, const double *omega, int n_w, double beta,
                double density, const double *S_bar, double *chi00_bar, double *beta_bar,
                tdx_stream stream);

/* chi00 = [A^{-1} chi0 e]_{g0}, A = 1 - chi0 K.  The cotangent of chi0(w)
 * is the rank-1 matrix u(w) v(w)^H with u = chi00_bar conj(A^{-T} e) and
 * v = e + K A^{-1} chi0 e; u, v: device complex128 [n_w][n_g] (written).
 * work: tdx_dyson_work_bytes(n_g, n_w) bytes; info: device int [n_w],
 * 0 or the failing pivot column + 1 (u, v NaN for that frequency).
 * No allocation or synchronisation. */
int tdx_dyson_vjp(tdx_ctx *ctx, const double *chi0, const double *K, int n_g, int n_w,
                  int i_g0, const double *chi00_bar, double *u, double *v, void *work,
                  int *info, tdx_stream stream);

/* chi0 = pref sum_t w_t rho_t rho_t^H, w_t = df_t / (w - delta_t + i eta)
 * (a paired list: w_t = df_t [1/(w - delta_t + i eta) - 1/(w + delta_t + i eta)]),
 * with cotangent u v^H per frequency, for the transitions t_begin ..
 * t_end - 1.  P: their FP64 pair densities (TDX_PREC_FP64 layout, row 0 =
 * t_begin, e.g. from tdx_pair_density_range).  Writes, per transition (row
 * t - t_begin), the real cotangents
 *   w_bar: device FP64 [t_end - t_begin][3] = (df_bar, delta_bar, eta_bar_t),
 *   dL = sum_t df_bar d(df_t) + delta_bar d(delta_t) + eta_bar_t d(eta),
 * and, if rho_bar is not NULL, the pair-density cotangent rho_bar: device
 * complex128 [t_end - t_begin][ld], ld = n_g rounded up to 16.  With
 * lambda = pref (u^H rho_t) conj(v^H rho_t) each entry is Re sum_w lambda
 * dw_t/dx.  No allocation or synchronisation. */
int tdx_chi0_vjp(tdx_ctx *ctx, const tdx_translist *tl, int64_t t_begin, int64_t t_end,
                 const double *P, int n_g, const double *omega, int n_w, double eta, double pref,
                 const double *u, const double *v, double *w_bar, double *rho_bar,
                 tdx_stream stream);

/* From w_bar of one q (device FP64 [n_trans][3] as written by tdx_chi0_vjp
 * for the whole list): accumulates the occupation and eigenvalue cotangents
 * of the states (occ_bar, eps_bar: device [n_k][nb_max], +=) through
 * df_t = f_n(k) - f_m(k') and delta_t = eps_m(k') - eps_n(k), and
 * eta_bar (device [1], += sum_t eta_bar_t).  Synchronises. */
int tdx_weights_vjp(tdx_ctx *ctx, const tdx_states *st, const int qj[3], const tdx_translist *tl,
                    int64_t n_trans, const double *w_bar, double *occ_bar, double *eps_bar,
                    double *eta_bar, tdx_stream stream);

/* Occupations f = 1/(1 + e^{(eps - mu)/T}) with mu fixed by the electron
 * count, at the states' current temperature and mu (call tdx_occupations
 * for the q's temperature first).  Writes T_bar (device [1], the
 * occupation path only) and accumulates eps_bar (+=, through mu(eps)). */
int tdx_occupations_vjp(tdx_ctx *ctx, const tdx_states *st, const double *occ_bar,
                        double *eps_bar, double *T_bar, tdx_stream stream);

/* rho_t(G) = sum_G1 c*_nk(G1) c_mk'(G1 + G + G_s): accumulates the
 * orbital cotangents coef_bar (device complex128 [n_k][nb_max][npw_max],
 * +=) from rho_bar of the transitions t_begin .. t_end - 1 of one q (layout
 * of tdx_chi0_vjp, row 0 = t_begin), so that a list can be swept in blocks.
 * Per k of the range the cost is two dense complex products of
 * n_g x nb x nb x npw (the range's rho_bar scattered into an nb x nb matrix
 * per G), whatever the number of the k's transitions in the range: ranges
 * cut at k boundaries avoid repeating them.  Workspace: up to 2 GiB of
 * products plus nb_max^2 per response vector of a block.  Synchronises. */
int tdx_pair_density_vjp(tdx_ctx *ctx, const tdx_states *st, const int qj[3],
                         const tdx_translist *tl, int64_t t_begin, int64_t t_end,
                         const int *gbasis, int n_g, const double *rho_bar, double *coef_bar,
                         tdx_stream stream);

/* Shell-value gradient from the eigenvalue and orbital cotangents of the
 * kept bands: with H(k) rebuilt and fully diagonalised (all N_pw pairs),
 *   y_n = sum_{m not in the multiplet of n} psi_m <psi_m|cbar_n> / (eps_n - eps_m),
 *   v_bar_s = sum_kn Re (eps_bar_n psi_n + y_n)^H (dH/dv_s) psi_n,
 * dH/dv_s = [G - G' on shell s] sum_I e^{-i (G-G').R_I}.  Rotations inside
 * a kept multiplet leave the loss unchanged, so those pairs are dropped.
 * md must be the model the states were built from; v_bar: host
 * [n_shells] (written).  Synchronises. */
int tdx_potential_vjp(tdx_ctx *ctx, const tdx_model *md, const tdx_states *st,
                      const double *eps_bar, const double *coef_bar, double *v_bar,
                      tdx_stream stream);

/* The adiabatic kernel's share of the reverse pass (ALDA, Sec. A.1): K
 * depends on the density of the states, n(r_j) =
 * 2/(N_k Omega) sum_kn f_nk |u_nk(r_j)|^2, through
 * K[a][b] = 4 pi/|q+G_a|^2 delta_ab + (1/N_r) sum_j f_xc(n(r_j)) e^{-i(G_a-G_b).r_j},
 * and n on the occupations (so on T) and the orbitals (so on v).  Three
 * calls, per q then once:
 *   dyson_kernel_vjp -> kernel_matrix_vjp (per q, accumulating fxc_bar on
 *   the grid) -> density_vjp (once: occ_bar and coef_bar, which then join
 *   the RPA chain's occupations_vjp and potential_vjp). */

/* K_bar += sum_w p_w x_w^H with x_w = A^{-1} chi0 e and p_w = chi0(w)^H u_w,
 * u_w = chi00_bar conj(A^{-T} e) (the cotangent of K through chi00 =
 * [A^{-1} chi0 e]_{g0}, A = 1 - chi0 K).  K_bar: device complex128
 * [n_g][n_g] (+=).  Workspace from the context; synchronises; NUMERIC if a
 * Dyson matrix is singular. */
int tdx_dyson_kernel_vjp(tdx_ctx *ctx, const double *chi0, const double *K, int n_g, int n_w,
                         int i_g0, const double *chi00_bar, double *K_bar, tdx_stream stream);

/* fxc_bar[j] += (1/N_r) Re sum_ab conj(K_bar[a][b]) e^{-i(G_a - G_b).r_j}: the
 * cotangent of f_xc(r_j) from the ALDA part of K (the Coulomb part depends
 * on no parameter).  gbasis: device int [n_g][3] (the basis K was built on);
 * dens_grid: host [3], the grid of tdx_xc_kernel_grid; fxc_bar: device
 * [N_r] (+=), grid order (j_0 N_1 + j_1) N_2 + j_2.  Synchronises. */
int tdx_kernel_matrix_vjp(tdx_ctx *ctx, const tdx_states *st, const int *gbasis, int n_g,
                          const int dens_grid[3], const double *K_bar, double *fxc_bar,
                          tdx_stream stream);

/* From fxc_bar: nbar = fxc_bar f_xc'(n) (f_xc' = d^3(n eps_xc)/dn^3), then
 *   occ_bar[k][n] += 2/(N_k Omega) sum_j nbar_j |u_nk(r_j)|^2,
 *   coef_bar[k][n](G) += 2 (2/(N_k Omega)) f_nk sum_j nbar_j u_nk(r_j) e^{-iG.r_j}
 * over the bands the density sums (f >= 1e-20).  occ_bar: device
 * [n_k][nb_max] (+=); coef_bar: device complex128 [n_k][nb_max][npw_max]
 * (+=) or null (temperature and broadening only).  Synchronises. */
int tdx_density_vjp(tdx_ctx *ctx, const tdx_states *st, const int dens_grid[3],
                    const double *fxc_bar, double *occ_bar, double *coef_bar,
                    tdx_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* TDX_H */
