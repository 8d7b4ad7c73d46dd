// Reverse mode (vector-Jacobian products) of the response chain
//   occupations -> transitions -> pair densities -> chi0 -> Dyson -> S -> F
// with respect to the temperature T, the broadening eta and, through the
// orbitals, the potential.  Complex cotangents follow dL = Re(conj(zbar) dz).
// All arithmetic is FP64; every reduction runs in a fixed order, so results
// are bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"
#include "tables.h"

namespace tdx {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ inline f64x4 mfma64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kVjpWaves = 4;
constexpr int kVjpT = 16 * kVjpWaves;  // transitions per workgroup, 16 per wave
constexpr int kVjpSub = 4;             // 16-frequency subtiles per block
constexpr int kVjpW = 16 * kVjpSub;    // frequencies per block
constexpr int kVjpG = 32;              // response vectors per LDS chunk
constexpr int kVjpRow = kVjpG + 1;     // padded LDS row (complex)

// chi0 = pref sum_t w_t rho_t rho_t^H with w_t = df_t / (w - delta_t + i eta)
// (full list) or, for a time-reversal paired list, the combined weight
// w_t = df_t (r1 - r2), r1 = 1 / (w - delta_t + i eta), r2 = 1 / (w + delta_t + i eta),
// and the cotangent of chi0(w) given as u(w) v(w)^H.  Then
//   dL = Re sum_w sum_t pref [dw_t alpha conj(beta)
//                             + w_t ((u^H d rho) conj(beta) + alpha conj(v^H d rho))],
// alpha = u^H rho_t, beta = v^H rho_t.  With lambda = pref alpha conj(beta),
//   full:   dw = r1 d(df) + df r1^2 d(delta) - i df r1^2 d(eta),
//   paired: dw = (r1 - r2) d(df) + df (r1^2 + r2^2) d(delta) - i df (r1^2 - r2^2) d(eta),
// so each transition's real cotangents are
//   wbar_t = (dfbar, deltabar, etabar_t)
//          = (Re sum_w lambda dw/d(df), Re sum_w lambda dw/d(delta), Re sum_w lambda dw/d(eta)),
// and rhobar_t(G) = sum_w conj(c1) u_G + c2 v_G with c1 = pref w_t conj(beta),
// c2 = pref w_t alpha.
__global__ void __launch_bounds__(256)
    k_chi0_vjp(const double2 *P, int ld, long long t_lo, long long n_trans, int n_g,
               const double *delta, const double *df, int paired, const double *omega, int n_w,
               double eta, double pref, const double2 *u, const double2 *v, double *wbar,
               double2 *rhobar) {
  // rows of P, wbar and rhobar are local (row i is transition t_lo + i)
  __shared__ double2 xs[2][kVjpW][kVjpRow];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, quad = lane >> 4;
  const long long tw0 = (long long)blockIdx.x * kVjpT + wave * 16;
  const long long t = tw0 + col;
  const long long tc = t < n_trans ? t : n_trans - 1;
  const double2 *prow = P + (size_t)tc * ld;
  const double dl = delta[t_lo + tc], dft = df[t_lo + tc];
  // sums of lambda times dw/d(df), dw/d(delta) / df, i dw/d(eta) / df
  double sfr = 0.0, sfi = 0.0, sdr = 0.0, sdi = 0.0, ser = 0.0, sei = 0.0;
  for (int w0 = 0; w0 < n_w; w0 += kVjpW) {
    f64x4 acc[kVjpSub][2][2];
#pragma unroll
    for (int sub = 0; sub < kVjpSub; ++sub)
#pragma unroll
      for (int x = 0; x < 2; ++x) acc[sub][x][0] = acc[sub][x][1] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int g0 = 0; g0 < ld; g0 += kVjpG) {
      __syncthreads();
      for (int e = threadIdx.x; e < 2 * kVjpW * kVjpG; e += 256) {
        const int mtx = e / (kVjpW * kVjpG), r = (e / kVjpG) % kVjpW, c = e % kVjpG;
        const int wi = w0 + r, gi = g0 + c;
        double2 x = make_double2(0.0, 0.0);
        if (wi < n_w && gi < n_g) {
          x = (mtx ? v : u)[(size_t)wi * n_g + gi];
          x.y = -x.y;
        }
        xs[mtx][r][c] = x;
      }
      __syncthreads();
      const int gn = min(kVjpG, ld - g0);
      for (int gs = 0; gs < gn; gs += 16) {
        double2 b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) b[i] = prow[g0 + gs + 4 * quad + i];
#pragma unroll
        for (int sub = 0; sub < kVjpSub; ++sub)
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const double2 a = xs[x][16 * sub + col][gs + 4 * quad + i];
              acc[sub][x][0] = mfma64(a.x, b[i].x, acc[sub][x][0]);
              acc[sub][x][0] = mfma64(-a.y, b[i].y, acc[sub][x][0]);
              acc[sub][x][1] = mfma64(a.x, b[i].y, acc[sub][x][1]);
              acc[sub][x][1] = mfma64(a.y, b[i].x, acc[sub][x][1]);
            }
      }
    }
    // epilogue: lane holds frequency w0 + 16 sub + quad + 4 j, transition t
#pragma unroll
    for (int sub = 0; sub < kVjpSub; ++sub)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int wi = w0 + 16 * sub + quad + 4 * j;
        const double ar = acc[sub][0][0][j], ai = acc[sub][0][1][j];
        const double br = acc[sub][1][0][j], bi = acc[sub][1][1][j];
        double c1r = 0.0, c1i = 0.0, c2r = 0.0, c2i = 0.0;
        if (wi < n_w) {
          const double lr = pref * (ar * br + ai * bi), li = pref * (ai * br - ar * bi);
          const double dr = omega[wi] - dl;
          const double inv = 1.0 / (dr * dr + eta * eta);
          // r1 = 1 / (w - delta + i eta) and its square
          const double r1r = dr * inv, r1i = -eta * inv;
          const double q1r = r1r * r1r - r1i * r1i, q1i = 2.0 * r1r * r1i;
          double gr = r1r, gi = r1i, hr = q1r, hi = q1i, er = q1r, ei = q1i;
          if (paired) {
            // r2 = 1 / (w + delta + i eta): g = r1 - r2, h = r1^2 + r2^2, e = r1^2 - r2^2
            const double d2 = omega[wi] + dl;
            const double inv2 = 1.0 / (d2 * d2 + eta * eta);
            const double r2r = d2 * inv2, r2i = -eta * inv2;
            const double q2r = r2r * r2r - r2i * r2i, q2i = 2.0 * r2r * r2i;
            gr = r1r - r2r;
            gi = r1i - r2i;
            hr = q1r + q2r;
            hi = q1i + q2i;
            er = q1r - q2r;
            ei = q1i - q2i;
          }
          sfr += lr * gr - li * gi;
          sfi += lr * gi + li * gr;
          sdr += lr * hr - li * hi;
          sdi += lr * hi + li * hr;
          ser += lr * er - li * ei;
          sei += lr * ei + li * er;
          const double wr = dft * gr, wim = dft * gi;
          c1r = pref * (wr * br + wim * bi);
          c1i = pref * (wim * br - wr * bi);
          c2r = pref * (wr * ar - wim * ai);
          c2i = pref * (wr * ai + wim * ar);
        }
        acc[sub][0][0][j] = c1r;
        acc[sub][0][1][j] = c1i;
        acc[sub][1][0][j] = c2r;
        acc[sub][1][1][j] = c2i;
      }
    if (rhobar) {
      for (int gc = 0; gc < ld; gc += 16) {
        f64x4 orr = {0.0, 0.0, 0.0, 0.0}, oi = {0.0, 0.0, 0.0, 0.0};
        const int gi = gc + col;
#pragma unroll
        for (int sub = 0; sub < kVjpSub; ++sub)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int wi = w0 + 16 * sub + 4 * j + quad;
            double2 uu = make_double2(0.0, 0.0), vv = make_double2(0.0, 0.0);
            if (wi < n_w && gi < n_g) {
              uu = u[(size_t)wi * n_g + gi];
              vv = v[(size_t)wi * n_g + gi];
            }
            const double c1r = acc[sub][0][0][j], c1i = acc[sub][0][1][j];
            const double c2r = acc[sub][1][0][j], c2i = acc[sub][1][1][j];
            orr = mfma64(c1r, uu.x, orr);
            orr = mfma64(c1i, uu.y, orr);
            orr = mfma64(c2r, vv.x, orr);
            orr = mfma64(-c2i, vv.y, orr);
            oi = mfma64(c1r, uu.y, oi);
            oi = mfma64(-c1i, uu.x, oi);
            oi = mfma64(c2r, vv.y, oi);
            oi = mfma64(c2i, vv.x, oi);
          }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const long long tr = tw0 + quad + 4 * j;
          if (tr < n_trans) {
            double2 *dst = rhobar + (size_t)tr * ld + gc + col;
            if (w0 == 0) {
              *dst = make_double2(orr[j], oi[j]);
            } else {
              double2 o = *dst;
              o.x += orr[j];
              o.y += oi[j];
              *dst = o;
            }
          }
        }
      }
    }
  }
  // lanes of one column hold disjoint frequencies of the same transition
  sfr += __shfl_xor(sfr, 16);
  sdr += __shfl_xor(sdr, 16);
  sei += __shfl_xor(sei, 16);
  sfr += __shfl_xor(sfr, 32);
  sdr += __shfl_xor(sdr, 32);
  sei += __shfl_xor(sei, 32);
  (void)sfi;
  (void)sdi;
  (void)ser;
  if (quad == 0 && t < n_trans) {
    // dw/d(eta) = -i df e, so Re(lambda dw/d(eta)) = df Im(sum lambda e)
    wbar[3 * t] = sfr;
    wbar[3 * t + 1] = dft * sdr;
    wbar[3 * t + 2] = dft * sei;
  }
}

// Per-state cotangents of one q from the transition cotangents
// wbar_t = (dfbar_t, deltabar_t, etabar_t):
//   occ_bar(k,n) += sum_{t out of (k,n)} dfbar_t,
//   occ_bar(k',m) -= sum_{t into (k',m)} dfbar_t,
//   eps_bar(k',m) += sum_{t into} deltabar_t, eps_bar(k,n) -= sum_{t out} deltabar_t.
// One thread per state; incoming transitions are found by binary search of
// m in each row of the source k-point (rows are sorted by m).
__global__ void k_weights_states(const double *wbar, const int *tm,
                                 const long long *rowbeg, const long long *rowend, const int *nb,
                                 const int *kinv, int nk, int nb_max, double *occ_bar,
                                 double *eps_bar) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)nk * nb_max) return;
  const int k = (int)(i / nb_max), j = (int)(i % nb_max);
  if (j >= nb[k]) return;
  double fb = 0.0, eb = 0.0;
  for (long long t = rowbeg[i]; t < rowend[i]; ++t) {
    fb += wbar[3 * t];
    eb -= wbar[3 * t + 1];
  }
  const int k0 = kinv[k];
  for (int n = 0; n < nb[k0]; ++n) {
    long long lo = rowbeg[(size_t)k0 * nb_max + n];
    const long long end = rowend[(size_t)k0 * nb_max + n];
    long long hi = end;
    while (lo < hi) {
      const long long mid = (lo + hi) >> 1;
      if (tm[mid] < j)
        lo = mid + 1;
      else
        hi = mid;
    }
    if (lo < end && tm[lo] == j) {
      fb -= wbar[3 * lo];
      eb += wbar[3 * lo + 1];
    }
  }
  occ_bar[i] += fb;
  eps_bar[i] += eb;
}

constexpr int kRedBlocks = 512;

// etabar = sum_t etabar_t: per-block partial sums over a fixed grid, then
// one fixed-order final sum.
__global__ void __launch_bounds__(256)
    k_eta_partial(const double *wbar, long long n, double *part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (long long t = blockIdx.x * 256LL + threadIdx.x; t < n; t += 256LL * kRedBlocks)
    acc += wbar[3 * t + 2];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) k_sum_into(const double *part, int n, double *out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] += sh[0];
}

// Occupations f_j = 1/(1 + e^{x_j}), x_j = (eps_j - mu)/T, with mu fixed by
// the electron count.  With w_j = f_j (1 - f_j):
//   mu_T = -(1/T) sum w (eps - mu) / sum w,   d mu / d eps_j = w_j / sum w,
//   Tbar = sum_j fbar_j w_j [(eps_j - mu)/T^2 + mu_T / T],
//   eps_bar_j += (w_j / T) (-fbar_j + sum_i fbar_i w_i / sum w).
constexpr int kOccThreads = 1024;

__device__ double block_sum1024(double x, double *sh) {
  sh[threadIdx.x] = x;
  __syncthreads();
  for (int s = kOccThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(kOccThreads)
    k_occ_vjp(const double *eps, const double *occ, const int *nb, int nk, int nb_max, double mu,
              double T, const double *occ_bar, double *eps_bar, double *T_bar) {
  __shared__ double sh[kOccThreads];
  double W = 0.0, We = 0.0, Wf = 0.0, Wfe = 0.0;
  const long tot = (long)nk * nb_max;
  for (long i = threadIdx.x; i < tot; i += kOccThreads) {
    if ((int)(i % nb_max) >= nb[i / nb_max]) continue;
    const double f = occ[i], w = f * (1.0 - f), e = eps[i] - mu, fb = occ_bar[i];
    W += w;
    We += w * e;
    Wf += fb * w;
    Wfe += fb * w * e;
  }
  W = block_sum1024(W, sh);
  We = block_sum1024(We, sh);
  Wf = block_sum1024(Wf, sh);
  Wfe = block_sum1024(Wfe, sh);
  const double muT = W > 0.0 ? -We / W / T : 0.0;
  const double mean = W > 0.0 ? Wf / W : 0.0;
  if (threadIdx.x == 0) T_bar[0] = Wfe / (T * T) + muT * Wf / T;
  for (long i = threadIdx.x; i < tot; i += kOccThreads) {
    if ((int)(i % nb_max) >= nb[i / nb_max]) continue;
    const double f = occ[i], w = f * (1.0 - f);
    eps_bar[i] += w / T * (mean - occ_bar[i]);
  }
}

// Pair-density adjoint by dense products, per k of the transition range and
// block of response vectors G_g (g0 <= g < g0 + gB):
//   S[g][m][n] = rhobar_(k,n,m)(G_g), zero where (k, n, m) is not in the range,
//   out: Mt[g][n][j] = sum_m conj(S[g][m][n]) c_{m k'}(j)           (zgemm N, C)
//        coef_bar(k, n)(G1) += sum_g Mt[g][n][L_k'(G1 + G_g + G_s)]
//   in:  Nt[g][m][i] = sum_n c_{n k}(i) S[g][m][n]                   (zgemm N, N)
//        coef_bar(k', m)(G2) += sum_g Nt[g][m][L_k(G2 - G_g - G_s)]
// which is
//   coef_bar(k,n)(G1) += sum_t sum_G conj(rhobar_t(G)) c_{m_t,k'}(G1 + G + G_s),
//   coef_bar(k',m)(G2) += sum_{n: (k,n,m)} sum_G rhobar_t(G) c_{n,k}(G2 - G - G_s)
// with the products on the MFMA (rocBLAS) and one lookup per (band, plane
// wave, G) instead of one per (transition, plane wave, G).

// S entries of the transitions [t0, t1) of one k (value = rhobar, or zero to
// clear them again after use).
__global__ void k_pdv_scatter(const int *tn, const int *tm, long long t0, long long t1,
                              long long t_lo, const double2 *rhobar, int ld, int g0, int n_g,
                              int nb_max, bool clear, double2 *S) {
  const long long t = t0 + blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int g = blockIdx.y;
  if (t >= t1 || g0 + g >= n_g) return;
  S[(size_t)g * nb_max * nb_max + (size_t)tm[t] * nb_max + tn[t]] =
      clear ? make_double2(0.0, 0.0) : rhobar[(size_t)(t - t_lo) * ld + g0 + g];
}

// coef_bar(k, b)(p) += sum_g X[g][b][lut(miller_k(p) + sg G_g + G_s)] for the
// bands b < nb of k and plane waves p < npw of k (sg = +1: outgoing side with
// the lookup of k'; sg = -1: incoming side, G_s negated by the caller, with
// the lookup of k).
__global__ void __launch_bounds__(256)
    k_pdv_gather(const double2 *X, int npw_max, int nb_max, int gB, int g0, const int *gbasis,
                 int sg, const int *mk, int npw, int nb, int s0, int s1, int s2, const int *lut,
                 int M0, int M1, int M2, double2 *cbar) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
  if (p >= npw || b >= nb) return;
  const int W1 = 2 * M1 + 1, W2 = 2 * M2 + 1;
  double ar = 0.0, ai = 0.0;
  for (int g = 0; g < gB; ++g) {
    const int *G = gbasis + 3 * (g0 + g);
    const int x0 = mk[3 * p] + sg * G[0] + s0 + M0;
    const int x1 = mk[3 * p + 1] + sg * G[1] + s1 + M1;
    const int x2 = mk[3 * p + 2] + sg * G[2] + s2 + M2;
    if (x0 < 0 || x0 > 2 * M0 || x1 < 0 || x1 >= W1 || x2 < 0 || x2 >= W2) continue;
    const int j = lut[((long)x0 * W1 + x1) * W2 + x2];
    if (j < 0) continue;
    const double2 v = X[((size_t)g * nb_max + b) * npw_max + j];
    ar += v.x;
    ai += v.y;
  }
  double2 &o = cbar[(size_t)b * npw_max + p];
  o.x += ar;
  o.y += ai;
}

// S_i = -Im chi_{j(i)} g_i(beta): j(i) = i, g = 1/(pi n (1 - e^{-beta w})) for
// w_i != 0; j(i) = i + 1, g = 1/(pi n beta w_{i+1}) at w_i = 0.
//   chi00_bar_j = i * (-sum_{i: j(i) = j} g_i Sbar_i),
//   beta_bar = sum_i Sbar_i (-Im chi_{j(i)}) dg_i/dbeta.
__global__ void __launch_bounds__(256)
    k_dsf_vjp(const double2 *chi, const double *w, int n, double beta, double dens,
              const double *Sbar, double2 *chi_bar, double *beta_bar) {
  __shared__ double sh[256];
  double bb = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) {
    double im = 0.0;
    if (w[j] != 0.0) {
      const double om = -expm1(-beta * w[j]);
      const double g = 1.0 / (M_PI * dens * om);
      im -= g * Sbar[j];
      const double dg = -w[j] * (1.0 - om) / (M_PI * dens * om * om);
      bb += Sbar[j] * (-chi[j].y) * dg;
    }
    if (j > 0 && w[j - 1] == 0.0) {
      const double g = 1.0 / (M_PI * dens * beta * w[j]);
      im -= g * Sbar[j - 1];
      bb += Sbar[j - 1] * (-chi[j].y) * (-g / beta);
    }
    chi_bar[j] = make_double2(0.0, im);
  }
  sh[threadIdx.x] = bb;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) beta_bar[0] = sh[0];
}

// F_j = sum_i c_i S_i (e^{-tau_j w_i} + e^{-(beta - tau_j) w_i}):
//   Sbar_i = c_i sum_j Fbar_j (e^{-tau_j w_i} + e^{-(beta - tau_j) w_i}),
//   tau_bar_j = Fbar_j sum_i c_i S_i w_i (e^{-(beta - tau_j) w_i} - e^{-tau_j w_i}),
//   beta_bar = -sum_j Fbar_j sum_i c_i S_i w_i e^{-(beta - tau_j) w_i}.
__device__ inline double trap_weight(const double *w, int n, int i) {
  double c = 0.0;
  if (i > 0) c += 0.5 * (w[i] - w[i - 1]);
  if (i + 1 < n) c += 0.5 * (w[i + 1] - w[i]);
  return c;
}

__global__ void __launch_bounds__(256)
    k_itcf_vjp(const double *S, const double *w, int n, double beta, const double *tau, int ntau,
               const double *Fbar, double *Sbar, double *tau_bar, double *beta_bar) {
  __shared__ double sa[256], sb[256];
  for (int i = threadIdx.x; i < n; i += 256) {
    double acc = 0.0;
    for (int j = 0; j < ntau; ++j)
      acc += Fbar[j] * (exp(-tau[j] * w[i]) + exp(-(beta - tau[j]) * w[i]));
    Sbar[i] = trap_weight(w, n, i) * acc;
  }
  double bsum = 0.0;
  for (int j = 0; j < ntau; ++j) {
    double ta = 0.0, tb = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
      const double cs = trap_weight(w, n, i) * S[i] * w[i];
      const double e1 = exp(-tau[j] * w[i]), e2 = exp(-(beta - tau[j]) * w[i]);
      ta += cs * (e2 - e1);
      tb += cs * e2;
    }
    sa[threadIdx.x] = ta;
    sb[threadIdx.x] = tb;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        sa[threadIdx.x] += sa[threadIdx.x + s];
        sb[threadIdx.x] += sb[threadIdx.x + s];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) tau_bar[j] = Fbar[j] * sa[0];
    bsum -= Fbar[j] * sb[0];
    __syncthreads();
  }
  if (threadIdx.x == 0) beta_bar[0] = bsum;
}

int ld_of(int n_g) { return (n_g + 15) / 16 * 16; }

// Lookup boxes, row ranges and k -> k' maps for one q (workspace slot WS_ADJ).
struct QTables {
  int *lut = nullptr;
  long long *rowbeg = nullptr, *rowend = nullptr;
  int *kp = nullptr, *gs = nullptr, *kinv = nullptr;
  long box = 0;
  double *part = nullptr;
};

int q_tables(tdx_ctx *ctx, const tdx_states *st, const int qj[3], const tdx_translist *tl,
             long long t_lo, long long t_hi, bool with_lut, hipStream_t s, QTables *q) {
  const int nk = st->n_k, nb_max = st->nb_max;
  const int M0 = st->mmax[0], M1 = st->mmax[1], M2 = st->mmax[2];
  q->box = (long)(2 * M0 + 1) * (2 * M1 + 1) * (2 * M2 + 1);
  const size_t lut_bytes = with_lut ? (sizeof(int) * (size_t)nk * q->box + 255) / 256 * 256 : 0;
  const size_t row_bytes = sizeof(long long) * 2 * (size_t)nk * nb_max;
  const size_t map_bytes = (sizeof(int) * 5 * (size_t)nk + 255) / 256 * 256;
  const size_t part_bytes = sizeof(double) * kRedBlocks;
  void *w;
  TDX_TRY(ws_get(ctx, WS_ADJ, lut_bytes + row_bytes + map_bytes + part_bytes, &w));
  char *p = (char *)w;
  q->lut = with_lut ? (int *)p : nullptr;
  q->rowbeg = (long long *)(p + lut_bytes);
  q->rowend = q->rowbeg + (size_t)nk * nb_max;
  q->kp = (int *)(p + lut_bytes + row_bytes);
  q->gs = q->kp + nk;
  q->kinv = q->gs + 3 * nk;
  q->part = (double *)(p + lut_bytes + row_bytes + map_bytes);
  std::vector<int> kp, gs, kinv(nk, 0);
  kq_map(st->kgrid, qj, &kp, &gs);
  for (int k = 0; k < nk; ++k) kinv[kp[k]] = k;
  TDX_HIP(hipMemcpyAsync(q->kp, kp.data(), sizeof(int) * nk, hipMemcpyHostToDevice, s));
  TDX_HIP(hipMemcpyAsync(q->gs, gs.data(), sizeof(int) * 3 * nk, hipMemcpyHostToDevice, s));
  TDX_HIP(hipMemcpyAsync(q->kinv, kinv.data(), sizeof(int) * nk, hipMemcpyHostToDevice, s));
  TDX_HIP(hipMemsetAsync(q->rowbeg, 0, row_bytes, s));
  hipLaunchKernelGGL(k_rows, dim3(nk), dim3(256), 0, s, (const long long *)tl->k_offsets, tl->n,
                     nb_max, t_lo, t_hi, q->rowbeg, q->rowend);
  TDX_HIP(hipGetLastError());
  if (with_lut) {
    TDX_HIP(hipMemsetAsync(q->lut, 0xff, lut_bytes, s));
    hipLaunchKernelGGL(k_lut, dim3((st->npw_max + 255) / 256, nk), dim3(256), 0, s, st->miller,
                       st->npw, st->npw_max, nk, M0, M1, M2, q->lut, q->box);
    TDX_HIP(hipGetLastError());
  }
  // the host vectors above are released on return: wait for their copies
  TDX_HIP(hipStreamSynchronize(s));
  return TDX_OK;
}

}  // namespace
}  // namespace tdx

using namespace tdx;

extern "C" {

int tdx_itcf_vjp(tdx_ctx *ctx, const double *S, const double *omega, int n_w, double beta,
                 const double *tau, int n_tau, const double *F_bar, double *S_bar,
                 double *tau_bar, double *beta_bar, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && S && omega && tau && F_bar && S_bar && tau_bar && beta_bar,
              TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_w > 0 && n_tau > 0, TDX_ERR_SHAPE, "bad sizes");
  TDX_REQUIRE(std::isfinite(beta) && beta > 0, TDX_ERR_INVALID_ARG, "bad beta");
  TDX_TRY(check_device(ctx));
  hipLaunchKernelGGL(k_itcf_vjp, dim3(1), dim3(256), 0, as_stream(stream), S, omega, n_w, beta,
                     tau, n_tau, F_bar, S_bar, tau_bar, beta_bar);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

int tdx_dsf_vjp(tdx_ctx *ctx, const double *chi00, const double *omega, int n_w, double beta,
                double density, const double *S_bar, double *chi00_bar, double *beta_bar,
                tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && chi00 && omega && S_bar && chi00_bar && beta_bar, TDX_ERR_INVALID_ARG,
              "null argument");
  TDX_REQUIRE(n_w > 0, TDX_ERR_SHAPE, "n_w must be positive");
  TDX_REQUIRE(std::isfinite(beta) && beta > 0 && std::isfinite(density) && density > 0,
              TDX_ERR_INVALID_ARG, "bad beta or density");
  TDX_TRY(check_device(ctx));
  hipLaunchKernelGGL(k_dsf_vjp, dim3(1), dim3(256), 0, as_stream(stream), (const double2 *)chi00,
                     omega, n_w, beta, density, S_bar, (double2 *)chi00_bar, beta_bar);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

int tdx_chi0_vjp(tdx_ctx *ctx, const tdx_translist *tl, int64_t t_begin, int64_t t_end,
                 const double *P, int n_g, const double *omega, int n_w, double eta, double pref,
                 const double *u, const double *v, double *w_bar, double *rho_bar,
                 tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && tl && P && omega && u && v && w_bar, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_g > 0 && n_w > 0 && t_begin >= 0 && t_begin <= t_end && t_end <= tl->capacity,
              TDX_ERR_SHAPE, "bad sizes");
  TDX_REQUIRE(std::isfinite(eta) && std::isfinite(pref), TDX_ERR_INVALID_ARG, "bad eta or pref");
  TDX_TRY(check_device(ctx));
  const long long n = t_end - t_begin;
  if (n == 0) return TDX_OK;
  const long long blocks = (n + kVjpT - 1) / kVjpT;
  TDX_REQUIRE(blocks <= 0x7fffffffLL, TDX_ERR_SHAPE, "too many transitions");
  hipLaunchKernelGGL(k_chi0_vjp, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream),
                     (const double2 *)P, ld_of(n_g), (long long)t_begin, n, n_g, tl->delta,
                     tl->df, (int)tl->paired, omega, n_w, eta, pref, (const double2 *)u,
                     (const double2 *)v, w_bar, (double2 *)rho_bar);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

int tdx_weights_vjp(tdx_ctx *ctx, const tdx_states *st, const int qj[3], const tdx_translist *tl,
                    int64_t n_trans, const double *w_bar, double *occ_bar, double *eps_bar,
                    double *eta_bar, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && st && qj && tl && w_bar && occ_bar && eps_bar && eta_bar,
              TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_trans >= 0 && n_trans <= tl->capacity, TDX_ERR_SHAPE, "bad sizes");
  TDX_TRY(check_device(ctx));
  if (n_trans == 0) return TDX_OK;
  hipStream_t s = as_stream(stream);
  QTables q;
  TDX_TRY(q_tables(ctx, st, qj, tl, 0, n_trans, false, s, &q));
  const long tot = (long)st->n_k * st->nb_max;
  hipLaunchKernelGGL(k_weights_states, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     w_bar, tl->m, q.rowbeg, q.rowend, st->nb, q.kinv, st->n_k, st->nb_max,
                     occ_bar, eps_bar);
  TDX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_eta_partial, dim3(kRedBlocks), dim3(256), 0, s, w_bar,
                     (long long)n_trans, q.part);
  TDX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(256), 0, s, q.part, kRedBlocks, eta_bar);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

int tdx_occupations_vjp(tdx_ctx *ctx, const tdx_states *st, const double *occ_bar,
                        double *eps_bar, double *T_bar, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && st && occ_bar && eps_bar && T_bar, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(std::isfinite(st->temperature) && st->temperature > 0, TDX_ERR_INVALID_ARG,
              "states carry no temperature");
  TDX_TRY(check_device(ctx));
  hipLaunchKernelGGL(k_occ_vjp, dim3(1), dim3(kOccThreads), 0, as_stream(stream), st->eps,
                     st->occ, st->nb, st->n_k, st->nb_max, st->mu, st->temperature, occ_bar,
                     eps_bar, T_bar);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

int tdx_pair_density_vjp(tdx_ctx *ctx, const tdx_states *st, const int qj[3],
                         const tdx_translist *tl, int64_t t_begin, int64_t t_end,
                         const int *gbasis, int n_g, const double *rho_bar, double *coef_bar,
                         tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && st && qj && tl && gbasis && rho_bar && coef_bar, TDX_ERR_INVALID_ARG,
              "null argument");
  TDX_REQUIRE(n_g > 0 && t_begin >= 0 && t_begin <= t_end && t_end <= tl->capacity,
              TDX_ERR_SHAPE, "bad sizes");
  TDX_TRY(check_device(ctx));
  if (t_end == t_begin) return TDX_OK;
  hipStream_t s = as_stream(stream);
  QTables q;
  TDX_TRY(q_tables(ctx, st, qj, tl, t_begin, t_end, true, s, &q));
  const int M0 = st->mmax[0], M1 = st->mmax[1], M2 = st->mmax[2];
  const int nk = st->n_k, nb_max = st->nb_max, npw_max = st->npw_max, ld = ld_of(n_g);
  // host copies of the per-k sizes, the k -> k' map and the list's k offsets
  std::vector<long long> koff(nk + 1);
  std::vector<int> nbh(nk), npwh(nk), kp, gs;
  TDX_HIP(hipMemcpyAsync(koff.data(), tl->k_offsets, sizeof(long long) * (nk + 1),
                         hipMemcpyDeviceToHost, s));
  TDX_HIP(hipMemcpyAsync(nbh.data(), st->nb, sizeof(int) * nk, hipMemcpyDeviceToHost, s));
  TDX_HIP(hipMemcpyAsync(npwh.data(), st->npw, sizeof(int) * nk, hipMemcpyDeviceToHost, s));
  TDX_HIP(hipStreamSynchronize(s));
  kq_map(st->kgrid, qj, &kp, &gs);
  // response vectors per block: the products of a block take at most 2 GiB
  const size_t per_g = (size_t)nb_max * npw_max * sizeof(double2);
  const int gB = (int)std::max<size_t>(1, std::min<size_t>(n_g, ((size_t)2 << 30) / per_g));
  const size_t s_bytes = ((size_t)gB * nb_max * nb_max * sizeof(double2) + 255) / 256 * 256;
  void *w;
  TDX_TRY(ws_get(ctx, WS_ADJ2, s_bytes + (size_t)gB * per_g, &w));
  double2 *S = (double2 *)w;
  double2 *X = (double2 *)((char *)w + s_bytes);
  const long long ns = (long long)gB * nb_max * nb_max;
  hipLaunchKernelGGL(k_fill<double2>, dim3((unsigned)std::min<long long>((ns + 255) / 256, 65535)),
                     dim3(256), 0, s, S, ns, make_double2(0.0, 0.0));
  TDX_HIP(hipGetLastError());
  TDX_REQUIRE(rocblas_set_stream(ctx->blas, s) == rocblas_status_success, TDX_ERR_HIP,
              "rocblas_set_stream failed");
  const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
  const double2 *coef = (const double2 *)st->coef;
  double2 *cbar = (double2 *)coef_bar;
  for (int k = 0; k < nk; ++k) {
    const long long t0 = std::max<long long>(koff[k], t_begin);
    const long long t1 = std::min<long long>(koff[k + 1], t_end);
    if (t1 <= t0) continue;
    const int k2 = kp[k];
    const int nb1 = nbh[k], nb2 = nbh[k2], np1 = npwh[k], np2 = npwh[k2];
    const double2 *c1 = coef + (size_t)k * nb_max * npw_max;
    const double2 *c2 = coef + (size_t)k2 * nb_max * npw_max;
    const dim3 sgrid((unsigned)((t1 - t0 + 255) / 256), gB);
    for (int g0 = 0; g0 < n_g; g0 += gB) {
      const int gb = std::min(gB, n_g - g0);
      hipLaunchKernelGGL(k_pdv_scatter, sgrid, dim3(256), 0, s, tl->n, tl->m, t0, t1,
                         (long long)t_begin, (const double2 *)rho_bar, ld, g0, n_g, nb_max, false,
                         S);
      TDX_HIP(hipGetLastError());
      // outgoing side: Mt = c_k'^T conj(S)^T, gathered into coef_bar(k, n)
      rocblas_status rs = rocblas_zgemm_strided_batched(
          ctx->blas, rocblas_operation_none, rocblas_operation_conjugate_transpose, np2, nb1, nb2,
          &one, (const rocblas_double_complex *)c2, npw_max, 0,
          (const rocblas_double_complex *)S, nb_max, (rocblas_stride)nb_max * nb_max, &zero,
          (rocblas_double_complex *)X, npw_max, (rocblas_stride)nb_max * npw_max, gb);
      TDX_REQUIRE(rs == rocblas_status_success, TDX_ERR_HIP, "rocblas_zgemm failed (%d)",
                  (int)rs);
      hipLaunchKernelGGL(k_pdv_gather, dim3((np1 + 255) / 256, nb1), dim3(256), 0, s, X, npw_max,
                         nb_max, gb, g0, gbasis, 1, st->miller + (size_t)k * npw_max * 3, np1,
                         nb1, gs[3 * k], gs[3 * k + 1], gs[3 * k + 2], q.lut + (size_t)k2 * q.box,
                         M0, M1, M2, cbar + (size_t)k * nb_max * npw_max);
      TDX_HIP(hipGetLastError());
      // incoming side: Nt = c_k^T S, gathered into coef_bar(k', m)
      rs = rocblas_zgemm_strided_batched(
          ctx->blas, rocblas_operation_none, rocblas_operation_none, np1, nb2, nb1, &one,
          (const rocblas_double_complex *)c1, npw_max, 0, (const rocblas_double_complex *)S,
          nb_max, (rocblas_stride)nb_max * nb_max, &zero, (rocblas_double_complex *)X, npw_max,
          (rocblas_stride)nb_max * npw_max, gb);
      TDX_REQUIRE(rs == rocblas_status_success, TDX_ERR_HIP, "rocblas_zgemm failed (%d)",
                  (int)rs);
      hipLaunchKernelGGL(k_pdv_gather, dim3((np2 + 255) / 256, nb2), dim3(256), 0, s, X, npw_max,
                         nb_max, gb, g0, gbasis, -1, st->miller + (size_t)k2 * npw_max * 3, np2,
                         nb2, -gs[3 * k], -gs[3 * k + 1], -gs[3 * k + 2],
                         q.lut + (size_t)k * q.box, M0, M1, M2,
                         cbar + (size_t)k2 * nb_max * npw_max);
      TDX_HIP(hipGetLastError());
      // S back to zero for the next block or k
      hipLaunchKernelGGL(k_pdv_scatter, sgrid, dim3(256), 0, s, tl->n, tl->m, t0, t1,
                         (long long)t_begin, (const double2 *)rho_bar, ld, g0, n_g, nb_max, true,
                         S);
      TDX_HIP(hipGetLastError());
    }
  }
  return TDX_OK;
}

}  // extern "C"
