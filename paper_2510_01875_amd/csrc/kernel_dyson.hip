// Interaction kernel K = v + f_xc and the Dyson solve, both FP64.
//
// K_GG' = 4 pi / |q+G|^2 delta_GG' + f_xc(G - G').  The ALDA part uses the
// density on the real-space grid r_j = sum_i (j_i/N_i) a_i,
//   n(r_j) = 2/(N_k Omega) sum_kn f_nk |sum_G c_nk(G) e^{i G.r_j}|^2,
// the local kernel f_xc(n) = d^2(n eps_xc)/dn^2 (Slater exchange + PW92
// correlation, Phys. Rev. B 45, 13244 (1992)), and
//   f_xc(G) = (1/N_r) sum_j f_xc(r_j) e^{-i G.r_j}.
// Both transforms are separable DFTs (three passes of 1D pencil sums with a
// twiddle table) on a box held in LDS.
//
// Dyson: chi = chi0 + chi0 K chi, column G0 by LU with partial pivoting of
// (1 - chi0 K), one workgroup per frequency.
#include <algorithm>
#include <climits>
#include <cmath>
#include <mutex>

#include "internal.h"

namespace tdx {
namespace {

constexpr int kMaxSide = 32;
constexpr double kOccSkip = 1e-20;

// One pass of 1D DFTs along `axis` of an N0 x N1 x N2 box in LDS (in place:
// each thread owns whole pencils).  sign = +1: sum_m x_m e^{+2 pi i m j/N}.
__device__ void dft_pass(double2 *box, const double2 *tw, int N0, int N1, int N2, int axis,
                         double sign) {
  const int Na = axis == 0 ? N0 : (axis == 1 ? N1 : N2);
  const int npen = N0 * N1 * N2 / Na;
  const int stride = axis == 0 ? N1 * N2 : (axis == 1 ? N2 : 1);
  for (int p = threadIdx.x; p < npen; p += blockDim.x) {
    int base;
    if (axis == 0) {
      base = p;  // p = i1 * N2 + i2
    } else if (axis == 1) {
      base = (p / N2) * N1 * N2 + (p % N2);
    } else {
      base = p * N2;
    }
    double2 v[kMaxSide];
    for (int m = 0; m < Na; ++m) v[m] = box[base + m * stride];
    for (int j = 0; j < Na; ++j) {
      double re = 0.0, im = 0.0;
      int idx = 0;  // (m * j) mod Na
      for (int m = 0; m < Na; ++m) {
        const double2 t = tw[idx];
        const double ti = sign * t.y;
        re = fma(v[m].x, t.x, fma(-v[m].y, ti, re));
        im = fma(v[m].x, ti, fma(v[m].y, t.x, im));
        idx += j;
        if (idx >= Na) idx -= Na;
      }
      box[base + j * stride] = make_double2(re, im);
    }
  }
}

// Twiddle tables for the three axes: tw + off[a], e^{2 pi i t / N_a}.
__device__ void make_twiddles(double2 *tw, int N0, int N1, int N2) {
  const int Ns[3] = {N0, N1, N2};
  int off = 0;
  for (int a = 0; a < 3; ++a) {
    for (int t = threadIdx.x; t < Ns[a]; t += blockDim.x) {
      double s, c;
      sincospi(2.0 * t / Ns[a], &s, &c);
      tw[off + t] = make_double2(c, s);
    }
    off += Ns[a];
  }
}

// Per-k density partial: dens[k][j] = sum_n f_nk |u_nk(r_j)|^2.
__global__ void __launch_bounds__(256)
    k_density(const double2 *coef, const double *occ, const int *nb, const int *npw,
              const int *miller, int nb_max, int npw_max, int N0, int N1, int N2,
              double *dens) {
  extern __shared__ double2 sm[];
  const int Nr = N0 * N1 * N2;
  double2 *box = sm;
  double2 *tw = sm + Nr;
  const int k = blockIdx.x;
  make_twiddles(tw, N0, N1, N2);
  double *out = dens + (size_t)k * Nr;
  for (int j = threadIdx.x; j < Nr; j += blockDim.x) out[j] = 0.0;
  const int nbk = nb[k], np = npw[k];
  const int *mk = miller + (size_t)k * npw_max * 3;
  for (int n = 0; n < nbk; ++n) {
    const double f = occ[(size_t)k * nb_max + n];
    if (!(f >= kOccSkip)) continue;
    __syncthreads();
    for (int j = threadIdx.x; j < Nr; j += blockDim.x) box[j] = make_double2(0.0, 0.0);
    __syncthreads();
    const double2 *c = coef + ((size_t)k * nb_max + n) * npw_max;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
      const int a = ((mk[3 * i] % N0) + N0) % N0;
      const int b = ((mk[3 * i + 1] % N1) + N1) % N1;
      const int d = ((mk[3 * i + 2] % N2) + N2) % N2;
      box[(a * N1 + b) * N2 + d] = c[i];
    }
    __syncthreads();
    dft_pass(box, tw + N0 + N1, N0, N1, N2, 2, 1.0);
    __syncthreads();
    dft_pass(box, tw + N0, N0, N1, N2, 1, 1.0);
    __syncthreads();
    dft_pass(box, tw, N0, N1, N2, 0, 1.0);
    __syncthreads();
    for (int j = threadIdx.x; j < Nr; j += blockDim.x) {
      const double2 u = box[j];
      out[j] = fma(f, u.x * u.x + u.y * u.y, out[j]);
    }
  }
}

__device__ void pw92(double rs, double *e, double *e1, double *e2) {
  const double A = 0.031091, a1 = 0.21370;
  const double b1 = 7.5957, b2 = 3.5876, b3 = 1.6382, b4 = 0.49294;
  const double s = sqrt(rs);
  const double Q = 2 * A * (b1 * s + b2 * rs + b3 * rs * s + b4 * rs * rs);
  const double Q1 = 2 * A * (0.5 * b1 / s + b2 + 1.5 * b3 * s + 2 * b4 * rs);
  const double Q2 = 2 * A * (-0.25 * b1 / (rs * s) + 0.75 * b3 / s + 2 * b4);
  const double L = log1p(1.0 / Q);
  const double D = Q + Q * Q;
  const double L1 = -Q1 / D;
  const double L2 = -Q2 / D + Q1 * Q1 * (1 + 2 * Q) / (D * D);
  const double g = -2 * A * (1 + a1 * rs);
  *e = g * L;
  *e1 = -2 * A * a1 * L + g * L1;
  *e2 = -4 * A * a1 * L1 + g * L2;
}

// Sum the per-k partials in k order, scale, apply f_xc(n) pointwise.
__global__ void k_fxc_real(const double *dens, int nk, int Nr, double scale, double2 *fx) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Nr) return;
  double s = 0.0;
  for (int k = 0; k < nk; ++k) s += dens[(size_t)k * Nr + j];
  const double n = s * scale;
  const double fxv = -(1.0 / 3.0) * cbrt(3.0 / M_PI) * pow(n, -2.0 / 3.0);
  const double rs = cbrt(3.0 / (4.0 * M_PI * n));
  double e, e1, e2;
  pw92(rs, &e, &e1, &e2);
  const double fcv = (rs * rs * e2 - 2.0 * rs * e1) / (9.0 * n);
  fx[j] = make_double2(fxv + fcv, 0.0);
}

// Third derivative of the PW92 correlation in rs (for the kernel's density
// response): with eps = g L(Q), g = -2A(1 + a1 rs) linear in rs,
//   d3 eps = 3 g' L2 + g L3,
//   L3 = -Q3/D + 3 Q1 Q2 (1 + 2Q)/D^2 + 2 Q1^3/D^2 - 2 Q1^3 (1 + 2Q)^2/D^3,
// D = Q(1 + Q), Qj and Lj the j-th derivatives in rs.
__device__ double pw92_e3(double rs) {
  const double A = 0.031091, a1 = 0.21370;
  const double b1 = 7.5957, b2 = 3.5876, b3 = 1.6382, b4 = 0.49294;
  const double s = sqrt(rs);
  const double Q = 2 * A * (b1 * s + b2 * rs + b3 * rs * s + b4 * rs * rs);
  const double Q1 = 2 * A * (0.5 * b1 / s + b2 + 1.5 * b3 * s + 2 * b4 * rs);
  const double Q2 = 2 * A * (-0.25 * b1 / (rs * s) + 0.75 * b3 / s + 2 * b4);
  const double Q3 = 2 * A * (0.375 * b1 / (rs * rs * s) - 0.375 * b3 / (rs * s));
  const double D = Q + Q * Q, T = 1 + 2 * Q;
  const double L2 = -Q2 / D + Q1 * Q1 * T / (D * D);
  const double L3 = -Q3 / D + 3 * Q1 * Q2 * T / (D * D) + 2 * Q1 * Q1 * Q1 / (D * D) -
                    2 * Q1 * Q1 * Q1 * T * T / (D * D * D);
  const double g = -2 * A * (1 + a1 * rs), g1 = -2 * A * a1;
  return 3 * g1 * L2 + g * L3;
}

// d f_xc / dn = d^3(n eps_xc)/dn^3: exchange (2/9)(3/pi)^(1/3) n^(-5/3);
// correlation, with f_c = (rs^2 e2 - 2 rs e1)/(9n) and d rs/dn = -rs/(3n),
//   d f_c/dn = -(rs^3 e3/3 + rs^2 e2 - (8/3) rs e1) / (9 n^2).
__device__ double fxc_deriv(double n) {
  const double dx = (2.0 / 9.0) * cbrt(3.0 / M_PI) * pow(n, -5.0 / 3.0);
  const double rs = cbrt(3.0 / (4.0 * M_PI * n));
  double e, e1, e2;
  pw92(rs, &e, &e1, &e2);
  const double e3 = pw92_e3(rs);
  const double dc =
      -(rs * rs * rs * e3 / 3.0 + rs * rs * e2 - (8.0 / 3.0) * rs * e1) / (9.0 * n * n);
  return dx + dc;
}

// Forward transform of f_xc on the box (one workgroup), scaled by 1/N_r.
__global__ void __launch_bounds__(256)
    k_fxc_forward(double2 *fx, int N0, int N1, int N2) {
  extern __shared__ double2 sm[];
  const int Nr = N0 * N1 * N2;
  double2 *box = sm, *tw = sm + Nr;
  make_twiddles(tw, N0, N1, N2);
  for (int j = threadIdx.x; j < Nr; j += blockDim.x) box[j] = fx[j];
  __syncthreads();
  dft_pass(box, tw + N0 + N1, N0, N1, N2, 2, -1.0);
  __syncthreads();
  dft_pass(box, tw + N0, N0, N1, N2, 1, -1.0);
  __syncthreads();
  dft_pass(box, tw, N0, N1, N2, 0, -1.0);
  __syncthreads();
  const double inv = 1.0 / Nr;
  for (int j = threadIdx.x; j < Nr; j += blockDim.x)
    fx[j] = make_double2(box[j].x * inv, box[j].y * inv);
}

__global__ void k_assemble_k(const int *gb, int n_g, double3 q, double3 b0, double3 b1,
                             double3 b2, const double2 *fxg, int N0, int N1, int N2, int alda,
                             double2 *K) {
  const int i = blockIdx.y, j = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_g || j >= n_g) return;
  double2 v = make_double2(0.0, 0.0);
  if (alda) {
    const int a = (((gb[3 * i] - gb[3 * j]) % N0) + N0) % N0;
    const int b = (((gb[3 * i + 1] - gb[3 * j + 1]) % N1) + N1) % N1;
    const int c = (((gb[3 * i + 2] - gb[3 * j + 2]) % N2) + N2) % N2;
    v = fxg[(a * N1 + b) * N2 + c];
  }
  if (i == j) {
    const int *m = gb + 3 * i;
    const double px = q.x + m[0] * b0.x + m[1] * b1.x + m[2] * b2.x;
    const double py = q.y + m[0] * b0.y + m[1] * b1.y + m[2] * b2.y;
    const double pz = q.z + m[0] * b0.z + m[1] * b1.z + m[2] * b2.z;
    v.x += 4.0 * M_PI / (px * px + py * py + pz * pz);
  }
  K[(size_t)i * n_g + j] = v;
}

// ------------------------------------------------------------------ Dyson
constexpr int kT = 16;

// A_w = I - chi0_w K (row-major), batched over w.
__global__ void k_one_minus(const double2 *chi0, const double2 *K, int n, double2 *A) {
  __shared__ double2 sa[kT][kT + 1], sb[kT][kT + 1];
  const int w = blockIdx.z;
  const int i = blockIdx.y * kT + threadIdx.y, j = blockIdx.x * kT + threadIdx.x;
  const double2 *C = chi0 + (size_t)w * n * n;
  double re = 0.0, im = 0.0;
  for (int l0 = 0; l0 < n; l0 += kT) {
    const int la = l0 + threadIdx.x, lb = l0 + threadIdx.y;
    sa[threadIdx.y][threadIdx.x] = (i < n && la < n) ? C[(size_t)i * n + la] : make_double2(0, 0);
    sb[threadIdx.y][threadIdx.x] = (lb < n && j < n) ? K[(size_t)lb * n + j] : make_double2(0, 0);
    __syncthreads();
#pragma unroll
    for (int l = 0; l < kT; ++l) {
      const double2 a = sa[threadIdx.y][l], b = sb[l][threadIdx.x];
      re = fma(a.x, b.x, fma(-a.y, b.y, re));
      im = fma(a.x, b.y, fma(a.y, b.x, im));
    }
    __syncthreads();
  }
  if (i < n && j < n)
    A[(size_t)w * n * n + (size_t)i * n + j] = make_double2((i == j ? 1.0 : 0.0) - re, -im);
}

constexpr int kLuThreads = 256;

__device__ inline double cabs1(double2 a) { return fabs(a.x) + fabs(a.y); }

__device__ inline double2 cdiv(double2 a, double2 b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  const double r = b.x / b.y, d = b.y + b.x * r;
  return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}

// LU with partial pivoting (largest |re|+|im|, lowest index on ties) of A_w,
// right-hand side chi0_w[:, g0]; writes x[g0] and a status per frequency.
__global__ void __launch_bounds__(kLuThreads)
    k_lu_solve(double2 *Aall, const double2 *chi0, int n, int g0, double2 *out, int *info) {
  extern __shared__ double2 sm[];
  double2 *b = sm;              // [n]
  double2 *l = sm + n;          // [n] multipliers
  __shared__ double pv[kLuThreads];
  __shared__ int pi[kLuThreads];
  __shared__ int fail;
  const int w = blockIdx.x, t = threadIdx.x;
  double2 *A = Aall + (size_t)w * n * n;
  const double2 *C = chi0 + (size_t)w * n * n;
  for (int i = t; i < n; i += kLuThreads) b[i] = C[(size_t)i * n + g0];
  if (t == 0) fail = 0;
  __syncthreads();
  for (int c = 0; c < n; ++c) {
    double best = -1.0;
    int arg = n;
    for (int r = c + t; r < n; r += kLuThreads) {
      const double v = cabs1(A[(size_t)r * n + c]);
      if (v > best) {
        best = v;
        arg = r;
      }
    }
    pv[t] = best;
    pi[t] = arg;
    __syncthreads();
    for (int s = kLuThreads / 2; s > 0; s >>= 1) {
      if (t < s) {
        if (pv[t + s] > pv[t] || (pv[t + s] == pv[t] && pi[t + s] < pi[t])) {
          pv[t] = pv[t + s];
          pi[t] = pi[t + s];
        }
      }
      __syncthreads();
    }
    const int p = pi[0];
    const double pmax = pv[0];
    if (!(pmax > 0.0) || !isfinite(pmax)) {
      if (t == 0) fail = c + 1;
      __syncthreads();
      break;
    }
    if (p != c) {
      for (int j = c + t; j < n; j += kLuThreads) {
        const double2 x = A[(size_t)c * n + j];
        A[(size_t)c * n + j] = A[(size_t)p * n + j];
        A[(size_t)p * n + j] = x;
      }
      if (t == 0) {
        const double2 x = b[c];
        b[c] = b[p];
        b[p] = x;
      }
    }
    __syncthreads();
    const double2 piv = A[(size_t)c * n + c];
    for (int r = c + 1 + t; r < n; r += kLuThreads) l[r] = cdiv(A[(size_t)r * n + c], piv);
    __syncthreads();
    const int m = n - c - 1;
    for (long e = t; e < (long)m * (m + 1); e += kLuThreads) {
      const int r = c + 1 + (int)(e / (m + 1));
      const int j = c + 1 + (int)(e % (m + 1));  // j == n stands for the right-hand side
      const double2 lr = l[r];
      if (j < n) {
        const double2 u = A[(size_t)c * n + j];
        double2 &a = A[(size_t)r * n + j];
        a.x = fma(-lr.x, u.x, fma(lr.y, u.y, a.x));
        a.y = fma(-lr.x, u.y, fma(-lr.y, u.x, a.y));
      } else {
        const double2 u = b[c];
        double2 &a = b[r];
        a.x = fma(-lr.x, u.x, fma(lr.y, u.y, a.x));
        a.y = fma(-lr.x, u.y, fma(-lr.y, u.x, a.y));
      }
    }
    __syncthreads();
  }
  if (fail) {
    if (t == 0) {
      info[w] = fail;
      out[w] = make_double2(NAN, NAN);
    }
    return;
  }
  // back substitution, x overwrites b
  __shared__ double sr[kLuThreads], si[kLuThreads];
  for (int r = n - 1; r >= 0; --r) {
    double re = 0.0, im = 0.0;
    for (int j = r + 1 + t; j < n; j += kLuThreads) {
      const double2 a = A[(size_t)r * n + j], x = b[j];
      re = fma(a.x, x.x, fma(-a.y, x.y, re));
      im = fma(a.x, x.y, fma(a.y, x.x, im));
    }
    sr[t] = re;
    si[t] = im;
    __syncthreads();
    for (int s = kLuThreads / 2; s > 0; s >>= 1) {
      if (t < s) {
        sr[t] += sr[t + s];
        si[t] += si[t + s];
      }
      __syncthreads();
    }
    if (t == 0) b[r] = cdiv(make_double2(b[r].x - sr[0], b[r].y - si[0]), A[(size_t)r * n + r]);
    __syncthreads();
  }
  if (t == 0) {
    info[w] = 0;
    out[w] = b[g0];
  }
}


// Reverse mode of the Dyson step.  chi_00 = e^T A^{-1} chi0 e with
// A = 1 - chi0 K (e = e_g0), so d chi_00 = a^T d chi0 b with
//   a = A^{-T} e            (row g0 of A^{-1}),
//   b = e + K x,  x = A^{-1} chi0 e   (column g0 of 1 + K chi).
// With the cotangent convention dL = Re(conj(cbar) d chi_00) the cotangent
// of chi0 is the rank-1 matrix u v^H, u = cbar conj(a), v = b.
// One workgroup per frequency: LU with partial pivoting of A in place (rows
// swapped whole, multipliers stored below the diagonal, pivot order kept),
// then U x = L^{-1} P chi0 e, and for a: U^T y = e, L^T z = y, a = P^T z.
__device__ inline void block_dot(double re, double im, double *sr, double *si) {
  const int t = threadIdx.x;
  sr[t] = re;
  si[t] = im;
  __syncthreads();
  for (int s = kLuThreads / 2; s > 0; s >>= 1) {
    if (t < s) {
      sr[t] += sr[t + s];
      si[t] += si[t + s];
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kLuThreads)
    k_lu_vjp(double2 *Aall, const double2 *chi0, const double2 *K, int n, int g0,
             const double2 *cbar, double2 *u, double2 *v, int *info, double2 *xout) {
  extern __shared__ double2 sm[];
  double2 *x = sm;                   // [n]
  double2 *y = sm + n;               // [n]
  int *piv = (int *)(sm + 2 * n);    // [n]
  __shared__ double pv[kLuThreads];
  __shared__ int pi[kLuThreads];
  __shared__ double sr[kLuThreads], si[kLuThreads];
  __shared__ int fail;
  const int w = blockIdx.x, t = threadIdx.x;
  double2 *A = Aall + (size_t)w * n * n;
  const double2 *C = chi0 + (size_t)w * n * n;
  for (int i = t; i < n; i += kLuThreads) x[i] = C[(size_t)i * n + g0];
  if (t == 0) fail = 0;
  __syncthreads();
  for (int c = 0; c < n; ++c) {
    double best = -1.0;
    int arg = n;
    for (int r = c + t; r < n; r += kLuThreads) {
      const double a = cabs1(A[(size_t)r * n + c]);
      if (a > best) {
        best = a;
        arg = r;
      }
    }
    pv[t] = best;
    pi[t] = arg;
    __syncthreads();
    for (int s = kLuThreads / 2; s > 0; s >>= 1) {
      if (t < s && (pv[t + s] > pv[t] || (pv[t + s] == pv[t] && pi[t + s] < pi[t]))) {
        pv[t] = pv[t + s];
        pi[t] = pi[t + s];
      }
      __syncthreads();
    }
    const int p = pi[0];
    const double pmax = pv[0];
    if (!(pmax > 0.0) || !isfinite(pmax)) {
      if (t == 0) fail = c + 1;
      __syncthreads();
      break;
    }
    if (t == 0) piv[c] = p;
    if (p != c) {
      for (int j = t; j < n; j += kLuThreads) {
        const double2 e = A[(size_t)c * n + j];
        A[(size_t)c * n + j] = A[(size_t)p * n + j];
        A[(size_t)p * n + j] = e;
      }
      if (t == 0) {
        const double2 e = x[c];
        x[c] = x[p];
        x[p] = e;
      }
    }
    __syncthreads();
    const double2 d = A[(size_t)c * n + c];
    for (int r = c + 1 + t; r < n; r += kLuThreads) A[(size_t)r * n + c] = cdiv(A[(size_t)r * n + c], d);
    __syncthreads();
    const int m = n - c - 1;
    for (long e = t; e < (long)m * (m + 1); e += kLuThreads) {
      const int r = c + 1 + (int)(e / (m + 1));
      const int j = c + 1 + (int)(e % (m + 1));  // j == n: right-hand side
      const double2 l = A[(size_t)r * n + c];
      const double2 src = j < n ? A[(size_t)c * n + j] : x[c];
      double2 &dst = j < n ? A[(size_t)r * n + j] : x[r];
      dst.x = fma(-l.x, src.x, fma(l.y, src.y, dst.x));
      dst.y = fma(-l.x, src.y, fma(-l.y, src.x, dst.y));
    }
    __syncthreads();
  }
  double2 *uw = u + (size_t)w * n, *vw = v + (size_t)w * n;
  if (fail) {
    for (int i = t; i < n; i += kLuThreads) uw[i] = vw[i] = make_double2(NAN, NAN);
    if (t == 0) info[w] = fail;
    return;
  }
  // U x = (L^{-1} P chi0 e), x overwritten
  for (int r = n - 1; r >= 0; --r) {
    double re = 0.0, im = 0.0;
    for (int j = r + 1 + t; j < n; j += kLuThreads) {
      const double2 a = A[(size_t)r * n + j], b = x[j];
      re = fma(a.x, b.x, fma(-a.y, b.y, re));
      im = fma(a.x, b.y, fma(a.y, b.x, im));
    }
    block_dot(re, im, sr, si);
    if (t == 0) x[r] = cdiv(make_double2(x[r].x - sr[0], x[r].y - si[0]), A[(size_t)r * n + r]);
    __syncthreads();
  }
  if (xout)
    for (int i = t; i < n; i += kLuThreads) xout[(size_t)w * n + i] = x[i];
  // v = e + K x
  for (int i = t; i < n; i += kLuThreads) {
    double re = i == g0 ? 1.0 : 0.0, im = 0.0;
    const double2 *Ki = K + (size_t)i * n;
    for (int j = 0; j < n; ++j) {
      const double2 a = Ki[j], b = x[j];
      re = fma(a.x, b.x, fma(-a.y, b.y, re));
      im = fma(a.x, b.y, fma(a.y, b.x, im));
    }
    vw[i] = make_double2(re, im);
  }
  // U^T y = e (forward), entries of U^T are A[j][i], j <= i
  for (int i = 0; i < n; ++i) {
    double re = 0.0, im = 0.0;
    for (int j = t; j < i; j += kLuThreads) {
      const double2 a = A[(size_t)j * n + i], b = y[j];
      re = fma(a.x, b.x, fma(-a.y, b.y, re));
      im = fma(a.x, b.y, fma(a.y, b.x, im));
    }
    block_dot(re, im, sr, si);
    if (t == 0)
      y[i] = cdiv(make_double2((i == g0 ? 1.0 : 0.0) - sr[0], -si[0]), A[(size_t)i * n + i]);
    __syncthreads();
  }
  // L^T z = y (backward, unit diagonal), z overwrites y
  for (int i = n - 1; i >= 0; --i) {
    double re = 0.0, im = 0.0;
    for (int j = i + 1 + t; j < n; j += kLuThreads) {
      const double2 a = A[(size_t)j * n + i], b = y[j];
      re = fma(a.x, b.x, fma(-a.y, b.y, re));
      im = fma(a.x, b.y, fma(a.y, b.x, im));
    }
    block_dot(re, im, sr, si);
    if (t == 0) y[i] = make_double2(y[i].x - sr[0], y[i].y - si[0]);
    __syncthreads();
  }
  // a = P^T z: undo the row swaps last to first
  if (t == 0) {
    for (int c = n - 1; c >= 0; --c) {
      const int p = piv[c];
      const double2 e = y[c];
      y[c] = y[p];
      y[p] = e;
    }
    info[w] = 0;
  }
  __syncthreads();
  const double2 cb = cbar[w];
  for (int i = t; i < n; i += kLuThreads) {
    const double2 a = y[i];  // u = cbar conj(a)
    uw[i] = make_double2(cb.x * a.x + cb.y * a.y, cb.y * a.x - cb.x * a.y);
  }
}

// ------------------------------------------------- ALDA kernel adjoint
// The cotangent of the kernel matrix from the Dyson solve, then of f_xc on
// the grid, then of the density and through it of the occupations and the
// orbitals.  With x = A^{-1} chi0 e, a = A^{-T} e and u = chi00_bar conj(a)
// (k_lu_vjp), d chi00 = (chi0^T a)^T dK x, so
//   Kbar[G][G'] = sum_w p_w[G] conj(x_w[G']),  p_w = chi0(w)^H u_w.

// p_w = chi0(w)^H u_w (row-major chi0: p[G] = sum_H conj(chi0[H][G]) u[H]).
__global__ void k_chi0h_u(const double2 *chi0, const double2 *u, int n, double2 *p) {
  const int w = blockIdx.y, g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const double2 *C = chi0 + (size_t)w * n * n;
  const double2 *uw = u + (size_t)w * n;
  double re = 0.0, im = 0.0;
  for (int h = 0; h < n; ++h) {
    const double2 c = C[(size_t)h * n + g], a = uw[h];
    re = fma(c.x, a.x, fma(c.y, a.y, re));
    im = fma(c.x, a.y, fma(-c.y, a.x, im));
  }
  p[(size_t)w * n + g] = make_double2(re, im);
}

// Kbar[G][G'] += sum_w p_w[G] conj(x_w[G']), frequencies in order.
__global__ void k_kbar(const double2 *p, const double2 *x, int n, int n_w, double2 *Kbar) {
  const int i = blockIdx.y, j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double re = 0.0, im = 0.0;
  for (int w = 0; w < n_w; ++w) {
    const double2 a = p[(size_t)w * n + i], b = x[(size_t)w * n + j];
    re = fma(a.x, b.x, fma(a.y, b.y, re));
    im = fma(a.y, b.x, fma(-a.x, b.y, im));
  }
  double2 &o = Kbar[(size_t)i * n + j];
  o.x += re;
  o.y += im;
}

// Phi[j][b] = exp(i G_b . r_j) = exp(2 pi i m_b . (j_0/N0, j_1/N1, j_2/N2)),
// the phases of the forward transform (integer products reduced mod N).
__global__ void k_phi(const int *gb, int n_g, int N0, int N1, int N2, double2 *Phi) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (b >= n_g) return;
  const int j0 = j / (N1 * N2), j1 = (j / N2) % N1, j2 = j % N2;
  const int p0 = ((gb[3 * b] * j0) % N0 + N0) % N0;
  const int p1 = ((gb[3 * b + 1] * j1) % N1 + N1) % N1;
  const int p2 = ((gb[3 * b + 2] * j2) % N2 + N2) % N2;
  double sn, cs;
  sincospi(2.0 * ((double)p0 / N0 + (double)p1 / N1 + (double)p2 / N2), &sn, &cs);
  Phi[(size_t)j * n_g + b] = make_double2(cs, sn);
}

// fbar[j] += (1/N_r) Re sum_a conj(Phi[j][a]) T[j][a], T[j][a] =
// sum_b conj(Kbar[a][b]) Phi[j][b]: the cotangent of f_xc(r_j) from
// K[a][b] = (1/N_r) sum_j f_xc(r_j) exp(-i (G_a - G_b) . r_j).
__global__ void k_fbar(const double2 *Phi, const double2 *T, int n_g, int Nr, double *fbar) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Nr) return;
  double re = 0.0;
  for (int a = 0; a < n_g; ++a) {
    const double2 f = Phi[(size_t)j * n_g + a], t = T[(size_t)j * n_g + a];
    re = fma(f.x, t.x, fma(f.y, t.y, re));
  }
  fbar[j] += re / Nr;
}

// nbar[j] = fbar[j] f_xc'(n(r_j)), n from the per-k partials in k order.
__global__ void k_nbar(const double *dens, int nk, int Nr, double scale, const double *fbar,
                       double *nbar) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Nr) return;
  double s = 0.0;
  for (int k = 0; k < nk; ++k) s += dens[(size_t)k * Nr + j];
  nbar[j] = fbar[j] * fxc_deriv(s * scale);
}

// Density adjoint per k (the bands the forward density summed):
//   occ_bar[k][n] += scale sum_j nbar_j |u_nk(r_j)|^2,
//   coef_bar[k][n](G) += 2 scale f_nk sum_j nbar_j u_nk(r_j) e^{-i G.r_j}
// (the second a forward transform of nbar u on the box, read at the basis).
__global__ void __launch_bounds__(256)
    k_density_vjp(const double2 *coef, const double *occ, const int *nb, const int *npw,
                  const int *miller, int nb_max, int npw_max, int N0, int N1, int N2,
                  double scale, const double *nbar, double *occ_bar, double2 *coef_bar) {
  extern __shared__ double2 sm[];
  __shared__ double red[256];
  const int Nr = N0 * N1 * N2;
  double2 *box = sm;
  double2 *tw = sm + Nr;
  const int k = blockIdx.x;
  make_twiddles(tw, N0, N1, N2);
  const int nbk = nb[k], np = npw[k];
  const int *mk = miller + (size_t)k * npw_max * 3;
  for (int n = 0; n < nbk; ++n) {
    const double f = occ[(size_t)k * nb_max + n];
    if (!(f >= kOccSkip)) continue;
    __syncthreads();
    for (int j = threadIdx.x; j < Nr; j += blockDim.x) box[j] = make_double2(0.0, 0.0);
    __syncthreads();
    const double2 *c = coef + ((size_t)k * nb_max + n) * npw_max;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
      const int a = ((mk[3 * i] % N0) + N0) % N0;
      const int b = ((mk[3 * i + 1] % N1) + N1) % N1;
      const int d = ((mk[3 * i + 2] % N2) + N2) % N2;
      box[(a * N1 + b) * N2 + d] = c[i];
    }
    __syncthreads();
    dft_pass(box, tw + N0 + N1, N0, N1, N2, 2, 1.0);
    __syncthreads();
    dft_pass(box, tw + N0, N0, N1, N2, 1, 1.0);
    __syncthreads();
    dft_pass(box, tw, N0, N1, N2, 0, 1.0);
    __syncthreads();
    double s = 0.0;
    for (int j = threadIdx.x; j < Nr; j += blockDim.x) {
      const double2 u = box[j];
      const double w = nbar[j];
      s = fma(w, u.x * u.x + u.y * u.y, s);
      box[j] = make_double2(w * u.x, w * u.y);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) occ_bar[(size_t)k * nb_max + n] += scale * red[0];
    if (coef_bar) {
      dft_pass(box, tw + N0 + N1, N0, N1, N2, 2, -1.0);
      __syncthreads();
      dft_pass(box, tw + N0, N0, N1, N2, 1, -1.0);
      __syncthreads();
      dft_pass(box, tw, N0, N1, N2, 0, -1.0);
      __syncthreads();
      double2 *cb = coef_bar + ((size_t)k * nb_max + n) * npw_max;
      const double g = 2.0 * scale * f;
      for (int i = threadIdx.x; i < np; i += blockDim.x) {
        const int a = ((mk[3 * i] % N0) + N0) % N0;
        const int b = ((mk[3 * i + 1] % N1) + N1) % N1;
        const int d = ((mk[3 * i + 2] % N2) + N2) % N2;
        const double2 v = box[(a * N1 + b) * N2 + d];
        cb[i].x += g * v.x;
        cb[i].y += g * v.y;
      }
    }
  }
}

// First failing frequency of a chunk of LU solves folded into the running
// status {frequency, column + 1} (one block; status[0] = INT_MAX: none yet).
__global__ void k_fold_status(const int *info, int n, int w0, int *status) {
  __shared__ int best[256];
  int b = INT_MAX;
  for (int i = threadIdx.x; i < n; i += 256)
    if (info[i] != 0) b = min(b, i);
  best[threadIdx.x] = b;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) best[threadIdx.x] = min(best[threadIdx.x], best[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && best[0] != INT_MAX && w0 + best[0] < status[0]) {
    status[0] = w0 + best[0];
    status[1] = info[best[0]];
  }
}

__global__ void k_clear_status(int *status) {
  if (threadIdx.x == 0) {
    status[0] = INT_MAX;
    status[1] = 0;
  }
}

// Scratch of the no-allocation Dyson entry point: a file-scope device array
// of fixed size (every GPU the library runs on holds its own copy until the
// process ends), laid out as the status words (256 bytes), the per-frequency
// pivot status of one chunk (rounded to 256 bytes), then the chunk's
// matrices 1 - chi0 K.  Host code reaches it only through the per-device
// address resolved below.
constexpr size_t kDysonScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kDysonScratchBytes];
void *g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mu;

size_t round256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

// With `device` current: resolve that device's address of the scratch array
// (once per device; later calls return at once).
int dyson_scratch_init(int device) {
  TDX_REQUIRE(device >= 0 && device < kMaxDevices, TDX_ERR_UNSUPPORTED,
              "device %d beyond the %d the scratch table holds", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return TDX_OK;
  void *p = nullptr;
  TDX_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  TDX_REQUIRE(p != nullptr, TDX_ERR_HIP, "no device address for the Dyson scratch");
  g_scratch_ptr[device] = p;
  return TDX_OK;
}

}  // namespace tdx

using namespace tdx;

extern "C" {

size_t tdx_dyson_noalloc_max_bytes(void) { return kDysonScratchBytes; }

int tdx_dyson_noalloc(tdx_ctx *ctx, const double *chi0, const double *K, int n_g, int n_w,
                      int i_g0, double *chi00, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && chi0 && K && chi00, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_g > 0 && n_w > 0 && i_g0 >= 0 && i_g0 < n_g, TDX_ERR_SHAPE, "bad sizes");
  TDX_REQUIRE((size_t)n_g * 2 * sizeof(double2) <= 64 * 1024, TDX_ERR_SHAPE,
              "n_g %d too large for the LU kernel", n_g);
  const size_t mat = sizeof(double2) * (size_t)n_g * n_g;
  // frequencies per pass: the status words, their pivot status and their
  // matrices must fit in the scratch
  long long cw = (long long)((kDysonScratchBytes - 512) / (mat + sizeof(int)));
  cw = std::min<long long>(std::min<long long>(cw, n_w), 65535);
  while (cw > 0 && 256 + round256(sizeof(int) * (size_t)cw) + mat * (size_t)cw > kDysonScratchBytes)
    --cw;
  TDX_REQUIRE(cw >= 1, TDX_ERR_SHAPE,
              "n_g %d: one %zu-byte matrix exceeds the %zu-byte scratch of this entry point", n_g,
              mat, kDysonScratchBytes);
  TDX_TRY(check_device(ctx));
  TDX_REQUIRE(ctx->device >= 0 && ctx->device < kMaxDevices && g_scratch_ptr[ctx->device],
              TDX_ERR_HIP, "scratch of device %d not set up", ctx->device);
  hipStream_t s = as_stream(stream);
  unsigned char *base = (unsigned char *)g_scratch_ptr[ctx->device];
  int *status = (int *)base;
  int *info = (int *)(base + 256);
  double2 *A = (double2 *)(base + 256 + round256(sizeof(int) * (size_t)cw));
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, status);
  TDX_HIP(hipGetLastError());
  const size_t n2 = (size_t)n_g * n_g;
  for (int w0 = 0; w0 < n_w; w0 += (int)cw) {
    const int nw = (int)std::min<long long>(cw, n_w - w0);
    const double2 *c = (const double2 *)chi0 + (size_t)w0 * n2;
    dim3 g((n_g + kT - 1) / kT, (n_g + kT - 1) / kT, nw);
    hipLaunchKernelGGL(k_one_minus, g, dim3(kT, kT), 0, s, c, (const double2 *)K, n_g, A);
    TDX_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_lu_solve, dim3(nw), dim3(kLuThreads), sizeof(double2) * 2 * n_g, s, A,
                       c, n_g, i_g0, (double2 *)chi00 + w0, info);
    TDX_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_fold_status, dim3(1), dim3(256), 0, s, info, nw, w0, status);
    TDX_HIP(hipGetLastError());
  }
  int h[2] = {0, 0};
  TDX_HIP(hipMemcpyAsync(h, status, sizeof(h), hipMemcpyDeviceToHost, s));
  TDX_HIP(hipStreamSynchronize(s));
  TDX_REQUIRE(h[0] == INT_MAX, TDX_ERR_NUMERIC,
              "Dyson matrix singular at frequency %d (column %d)", h[0], h[1] - 1);
  return TDX_OK;
}


// Check the density grid against the states and the LDS of the density and
// FFT kernels.
static int check_grid(const tdx_states *st, const int dens_grid[3], int *Nr, size_t *lds) {
  TDX_REQUIRE(dens_grid, TDX_ERR_INVALID_ARG, "ALDA needs a density grid");
  for (int i = 0; i < 3; ++i)
    TDX_REQUIRE(dens_grid[i] >= 2 * st->mmax[i] + 1 && dens_grid[i] <= kMaxSide, TDX_ERR_SHAPE,
                "density grid side %d must lie in [%d, %d]", dens_grid[i], 2 * st->mmax[i] + 1,
                kMaxSide);
  *Nr = dens_grid[0] * dens_grid[1] * dens_grid[2];
  *lds = sizeof(double2) * (*Nr + dens_grid[0] + dens_grid[1] + dens_grid[2]);
  TDX_REQUIRE(*lds <= 160 * 1024, TDX_ERR_SHAPE, "density grid of %d points exceeds LDS", *Nr);
  return TDX_OK;
}

int tdx_xc_kernel_grid(tdx_ctx *ctx, const tdx_states *st, const int dens_grid[3], double *fxg,
                       tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && st && fxg, TDX_ERR_INVALID_ARG, "null argument");
  TDX_TRY(check_device(ctx));
  int Nr;
  size_t lds;
  TDX_TRY(check_grid(st, dens_grid, &Nr, &lds));
  hipStream_t s = as_stream(stream);
  const int N0 = dens_grid[0], N1 = dens_grid[1], N2 = dens_grid[2];
  void *w;
  TDX_TRY(ws_get(ctx, WS_DENS, sizeof(double) * (size_t)st->n_k * Nr, &w));
  double *dens = (double *)w;
  TDX_HIP(hipFuncSetAttribute((const void *)k_density, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds));
  TDX_HIP(hipFuncSetAttribute((const void *)k_fxc_forward,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_density, dim3(st->n_k), dim3(256), lds, s, (const double2 *)st->coef,
                     st->occ, st->nb, st->npw, st->miller, st->nb_max, st->npw_max, N0, N1, N2,
                     dens);
  TDX_HIP(hipGetLastError());
  const double scale = 2.0 / (st->n_k * st->omega_cell);
  hipLaunchKernelGGL(k_fxc_real, dim3((Nr + 255) / 256), dim3(256), 0, s, dens, st->n_k, Nr,
                     scale, (double2 *)fxg);
  TDX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_fxc_forward, dim3(1), dim3(256), lds, s, (double2 *)fxg, N0, N1, N2);
  TDX_HIP(hipGetLastError());
  TDX_HIP(hipStreamSynchronize(s));  // the density workspace may be reused after return
  return TDX_OK;
}

int tdx_kernel_matrix_from_grid(tdx_ctx *ctx, const tdx_states *st, const int qj[3],
                                const int *gbasis, int n_g, int xc, const int dens_grid[3],
                                const double *fxg, double *K, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && st && qj && gbasis && K, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(xc == TDX_XC_RPA || xc == TDX_XC_ALDA, TDX_ERR_INVALID_ARG, "bad xc");
  TDX_REQUIRE(n_g > 0, TDX_ERR_SHAPE, "n_g must be positive");
  TDX_TRY(check_device(ctx));
  int N0 = 1, N1 = 1, N2 = 1;
  if (xc == TDX_XC_ALDA) {
    TDX_REQUIRE(fxg, TDX_ERR_INVALID_ARG, "ALDA needs the kernel grid");
    int Nr;
    size_t lds;
    TDX_TRY(check_grid(st, dens_grid, &Nr, &lds));
    N0 = dens_grid[0];
    N1 = dens_grid[1];
    N2 = dens_grid[2];
  }
  hipStream_t s = as_stream(stream);
  const double *B = st->bvec;
  const double3 b0 = make_double3(B[0], B[1], B[2]), b1 = make_double3(B[3], B[4], B[5]),
                b2 = make_double3(B[6], B[7], B[8]);
  double qr[3];
  for (int i = 0; i < 3; ++i) qr[i] = (double)qj[i] / st->kgrid[i];
  const double3 q = make_double3(qr[0] * B[0] + qr[1] * B[3] + qr[2] * B[6],
                                 qr[0] * B[1] + qr[1] * B[4] + qr[2] * B[7],
                                 qr[0] * B[2] + qr[1] * B[5] + qr[2] * B[8]);
  hipLaunchKernelGGL(k_assemble_k, dim3((n_g + 63) / 64, n_g), dim3(64), 0, s, gbasis, n_g, q, b0,
                     b1, b2, xc == TDX_XC_ALDA ? (const double2 *)fxg : nullptr, N0, N1, N2,
                     xc == TDX_XC_ALDA ? 1 : 0, (double2 *)K);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

int tdx_kernel_matrix(tdx_ctx *ctx, const tdx_states *st, const int qj[3], const int *gbasis,
                      int n_g, int xc, const int dens_grid[3], double *K, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && st && qj && gbasis && K, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(xc == TDX_XC_RPA || xc == TDX_XC_ALDA, TDX_ERR_INVALID_ARG, "bad xc");
  if (xc == TDX_XC_RPA)
    return tdx_kernel_matrix_from_grid(ctx, st, qj, gbasis, n_g, xc, dens_grid, nullptr, K,
                                       stream);
  int Nr;
  size_t lds;
  TDX_TRY(check_grid(st, dens_grid, &Nr, &lds));
  void *w;
  TDX_TRY(ws_get(ctx, WS_FXC, sizeof(double2) * (size_t)Nr, &w));
  TDX_TRY(tdx_xc_kernel_grid(ctx, st, dens_grid, (double *)w, stream));
  TDX_TRY(tdx_kernel_matrix_from_grid(ctx, st, qj, gbasis, n_g, xc, dens_grid, (const double *)w,
                                      K, stream));
  TDX_HIP(hipStreamSynchronize(as_stream(stream)));
  return TDX_OK;
}

size_t tdx_dyson_work_bytes(int n_g, int n_w) {
  return sizeof(double2) * (size_t)n_w * n_g * n_g;
}

int tdx_dyson_async(tdx_ctx *ctx, const double *chi0, const double *K, int n_g, int n_w,
                    int i_g0, double *chi00, void *work, int *info, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && chi0 && K && chi00 && work && info, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_g > 0 && n_w > 0 && i_g0 >= 0 && i_g0 < n_g, TDX_ERR_SHAPE, "bad sizes");
  TDX_REQUIRE((size_t)n_g * 2 * sizeof(double2) <= 64 * 1024, TDX_ERR_SHAPE,
              "n_g %d too large for the LU kernel", n_g);
  TDX_REQUIRE(n_w <= 65535, TDX_ERR_SHAPE, "n_w %d above 65535", n_w);
  hipStream_t s = as_stream(stream);
  double2 *A = (double2 *)work;
  dim3 g((n_g + kT - 1) / kT, (n_g + kT - 1) / kT, n_w);
  hipLaunchKernelGGL(k_one_minus, g, dim3(kT, kT), 0, s, (const double2 *)chi0,
                     (const double2 *)K, n_g, A);
  TDX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_lu_solve, dim3(n_w), dim3(kLuThreads), sizeof(double2) * 2 * n_g, s, A,
                     (const double2 *)chi0, n_g, i_g0, (double2 *)chi00, info);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

int tdx_dyson(tdx_ctx *ctx, const double *chi0, const double *K, int n_g, int n_w, int i_g0,
              double *chi00, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && chi0 && K && chi00, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_g > 0 && n_w > 0 && i_g0 >= 0 && i_g0 < n_g, TDX_ERR_SHAPE, "bad sizes");
  TDX_TRY(check_device(ctx));
  hipStream_t s = as_stream(stream);
  void *w;
  const size_t abytes = tdx_dyson_work_bytes(n_g, n_w);
  TDX_TRY(ws_get(ctx, WS_DYSON, abytes + sizeof(int) * n_w, &w));
  int *info = (int *)((char *)w + abytes);
  TDX_TRY(tdx_dyson_async(ctx, chi0, K, n_g, n_w, i_g0, chi00, w, info, stream));
  std::vector<int> h(n_w);
  TDX_HIP(hipMemcpyAsync(h.data(), info, sizeof(int) * n_w, hipMemcpyDeviceToHost, s));
  TDX_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < n_w; ++i)
    TDX_REQUIRE(h[i] == 0, TDX_ERR_NUMERIC, "Dyson matrix singular at frequency %d (column %d)",
                i, h[i] - 1);
  return TDX_OK;
}

int tdx_dyson_vjp(tdx_ctx *ctx, const double *chi0, const double *K, int n_g, int n_w, int i_g0,
                  const double *chi00_bar, double *u, double *v, void *work, int *info,
                  tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && chi0 && K && chi00_bar && u && v && work && info, TDX_ERR_INVALID_ARG,
              "null argument");
  TDX_REQUIRE(n_g > 0 && n_w > 0 && i_g0 >= 0 && i_g0 < n_g, TDX_ERR_SHAPE, "bad sizes");
  const size_t lds = (sizeof(double2) * 2 + sizeof(int)) * (size_t)n_g;
  TDX_REQUIRE(lds <= 64 * 1024, TDX_ERR_SHAPE, "n_g %d too large for the LU kernel", n_g);
  TDX_REQUIRE(n_w <= 65535, TDX_ERR_SHAPE, "n_w %d above 65535", n_w);
  hipStream_t s = as_stream(stream);
  double2 *A = (double2 *)work;
  dim3 g((n_g + kT - 1) / kT, (n_g + kT - 1) / kT, n_w);
  hipLaunchKernelGGL(k_one_minus, g, dim3(kT, kT), 0, s, (const double2 *)chi0,
                     (const double2 *)K, n_g, A);
  TDX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_lu_vjp, dim3(n_w), dim3(kLuThreads), lds, s, A, (const double2 *)chi0,
                     (const double2 *)K, n_g, i_g0, (const double2 *)chi00_bar, (double2 *)u,
                     (double2 *)v, info, (double2 *)nullptr);
  TDX_HIP(hipGetLastError());
  return TDX_OK;
}

int tdx_dyson_kernel_vjp(tdx_ctx *ctx, const double *chi0, const double *K, int n_g, int n_w,
                         int i_g0, const double *chi00_bar, double *K_bar, tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && chi0 && K && chi00_bar && K_bar, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_g > 0 && n_w > 0 && i_g0 >= 0 && i_g0 < n_g, TDX_ERR_SHAPE, "bad sizes");
  const size_t lds = (sizeof(double2) * 2 + sizeof(int)) * (size_t)n_g;
  TDX_REQUIRE(lds <= 64 * 1024, TDX_ERR_SHAPE, "n_g %d too large for the LU kernel", n_g);
  TDX_REQUIRE(n_w <= 65535 && n_g <= 65535, TDX_ERR_SHAPE, "sizes above the grid");
  TDX_TRY(check_device(ctx));
  hipStream_t s = as_stream(stream);
  const size_t mat = sizeof(double2) * (size_t)n_w * n_g * n_g;
  const size_t vec = sizeof(double2) * (size_t)n_w * n_g;
  const size_t ints = (sizeof(int) * ((size_t)n_w + 2) + 255) / 256 * 256;
  void *w;
  TDX_TRY(ws_get(ctx, WS_DYSON, mat + 4 * vec + ints, &w));
  double2 *A = (double2 *)w;
  double2 *u = (double2 *)((char *)w + mat), *v = u + (size_t)n_w * n_g;
  double2 *x = v + (size_t)n_w * n_g, *p = x + (size_t)n_w * n_g;
  int *info = (int *)(p + (size_t)n_w * n_g), *status = info + n_w;
  dim3 g((n_g + kT - 1) / kT, (n_g + kT - 1) / kT, n_w);
  hipLaunchKernelGGL(k_one_minus, g, dim3(kT, kT), 0, s, (const double2 *)chi0,
                     (const double2 *)K, n_g, A);
  TDX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_lu_vjp, dim3(n_w), dim3(kLuThreads), lds, s, A, (const double2 *)chi0,
                     (const double2 *)K, n_g, i_g0, (const double2 *)chi00_bar, u, v, info, x);
  TDX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, s, status);
  hipLaunchKernelGGL(k_fold_status, dim3(1), dim3(256), 0, s, info, n_w, 0, status);
  TDX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_chi0h_u, dim3((n_g + 63) / 64, n_w), dim3(64), 0, s, (const double2 *)chi0,
                     u, n_g, p);
  TDX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_kbar, dim3((n_g + 63) / 64, n_g), dim3(64), 0, s, p, x, n_g, n_w,
                     (double2 *)K_bar);
  TDX_HIP(hipGetLastError());
  int h[2] = {0, 0};
  TDX_HIP(hipMemcpyAsync(h, status, sizeof(h), hipMemcpyDeviceToHost, s));
  TDX_HIP(hipStreamSynchronize(s));
  TDX_REQUIRE(h[0] == INT_MAX, TDX_ERR_NUMERIC,
              "Dyson matrix singular at frequency %d (column %d)", h[0], h[1] - 1);
  return TDX_OK;
}

int tdx_kernel_matrix_vjp(tdx_ctx *ctx, const tdx_states *st, const int *gbasis, int n_g,
                          const int dens_grid[3], const double *K_bar, double *fxc_bar,
                          tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && st && gbasis && K_bar && fxc_bar, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(n_g > 0 && n_g <= 65535, TDX_ERR_SHAPE, "bad n_g");
  TDX_TRY(check_device(ctx));
  int Nr;
  size_t lds;
  TDX_TRY(check_grid(st, dens_grid, &Nr, &lds));
  hipStream_t s = as_stream(stream);
  const int N0 = dens_grid[0], N1 = dens_grid[1], N2 = dens_grid[2];
  const size_t mat = sizeof(double2) * (size_t)Nr * n_g;
  void *w;
  TDX_TRY(ws_get(ctx, WS_ADJ2, 2 * mat, &w));
  double2 *Phi = (double2 *)w, *T = (double2 *)((char *)w + mat);
  hipLaunchKernelGGL(k_phi, dim3((n_g + 63) / 64, Nr), dim3(64), 0, s, gbasis, n_g, N0, N1, N2,
                     Phi);
  TDX_HIP(hipGetLastError());
  TDX_REQUIRE(rocblas_set_stream(ctx->blas, s) == rocblas_status_success, TDX_ERR_HIP,
              "rocblas_set_stream failed");
  const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
  // T (column-major n_g x N_r) = Kbar_cm^H Phi_cm, Kbar_cm(b, a) = Kbar[a][b]
  const rocblas_status rs = rocblas_zgemm(
      ctx->blas, rocblas_operation_conjugate_transpose, rocblas_operation_none, n_g, Nr, n_g, &one,
      (const rocblas_double_complex *)K_bar, n_g, (const rocblas_double_complex *)Phi, n_g, &zero,
      (rocblas_double_complex *)T, n_g);
  TDX_REQUIRE(rs == rocblas_status_success, TDX_ERR_HIP, "rocblas_zgemm failed (%d)", (int)rs);
  hipLaunchKernelGGL(k_fbar, dim3((Nr + 255) / 256), dim3(256), 0, s, Phi, T, n_g, Nr, fxc_bar);
  TDX_HIP(hipGetLastError());
  TDX_HIP(hipStreamSynchronize(s));  // the workspace may be reused after return
  return TDX_OK;
}

int tdx_density_vjp(tdx_ctx *ctx, const tdx_states *st, const int dens_grid[3],
                    const double *fxc_bar, double *occ_bar, double *coef_bar,
                    tdx_stream stream) {
  clear_error();
  TDX_REQUIRE(ctx && st && fxc_bar && occ_bar, TDX_ERR_INVALID_ARG, "null argument");
  TDX_TRY(check_device(ctx));
  int Nr;
  size_t lds;
  TDX_TRY(check_grid(st, dens_grid, &Nr, &lds));
  TDX_REQUIRE(lds + 256 * sizeof(double) <= 160 * 1024, TDX_ERR_SHAPE,
              "density grid of %d points exceeds LDS", Nr);
  hipStream_t s = as_stream(stream);
  const int N0 = dens_grid[0], N1 = dens_grid[1], N2 = dens_grid[2];
  void *w;
  TDX_TRY(ws_get(ctx, WS_DENS, sizeof(double) * ((size_t)st->n_k + 1) * Nr, &w));
  double *dens = (double *)w, *nbar = dens + (size_t)st->n_k * Nr;
  TDX_HIP(hipFuncSetAttribute((const void *)k_density, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds));
  TDX_HIP(hipFuncSetAttribute((const void *)k_density_vjp,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_density, dim3(st->n_k), dim3(256), lds, s, (const double2 *)st->coef,
                     st->occ, st->nb, st->npw, st->miller, st->nb_max, st->npw_max, N0, N1, N2,
                     dens);
  TDX_HIP(hipGetLastError());
  const double scale = 2.0 / (st->n_k * st->omega_cell);
  hipLaunchKernelGGL(k_nbar, dim3((Nr + 255) / 256), dim3(256), 0, s, dens, st->n_k, Nr, scale,
                     fxc_bar, nbar);
  TDX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_density_vjp, dim3(st->n_k), dim3(256), lds, s, (const double2 *)st->coef,
                     st->occ, st->nb, st->npw, st->miller, st->nb_max, st->npw_max, N0, N1, N2,
                     scale, nbar, occ_bar, (double2 *)coef_bar);
  TDX_HIP(hipGetLastError());
  TDX_HIP(hipStreamSynchronize(s));  // the density workspace may be reused after return
  return TDX_OK;
}

}  // extern "C"
