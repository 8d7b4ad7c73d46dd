// Context, errors, workspaces and host geometry of the tdx library.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <numeric>

#include "internal.h"

namespace tdx {

static thread_local std::string g_error;

int fail(int code, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

void clear_error() { g_error.clear(); }

size_t ws_total(const tdx_ctx *ctx) {
  size_t s = 0;
  for (const auto &w : ctx->ws) s += w.bytes;
  return s;
}

int ws_get(tdx_ctx *ctx, int slot, size_t bytes, void **out) {
  Workspace &w = ctx->ws[slot];
  if (bytes <= w.bytes && w.ptr) {
    *out = w.ptr;
    return TDX_OK;
  }
  size_t grown = std::max(bytes, w.bytes + w.bytes / 4);
  if (ctx->limit && ws_total(ctx) - w.bytes + bytes > ctx->limit)
    return fail(TDX_ERR_ALLOC, "workspace of %zu bytes exceeds the context limit %zu",
                ws_total(ctx) - w.bytes + bytes, ctx->limit);
  if (ctx->limit && ws_total(ctx) - w.bytes + grown > ctx->limit) grown = bytes;
  if (w.ptr) {
    TDX_HIP(hipDeviceSynchronize());
    TDX_HIP(hipFree(w.ptr));
    w.ptr = nullptr;
    w.bytes = 0;
  }
  hipError_t e = hipMalloc(&w.ptr, grown);
  if (e != hipSuccess) {
    w.ptr = nullptr;
    return fail(TDX_ERR_ALLOC, "hipMalloc(%zu) failed: %s", grown, hipGetErrorString(e));
  }
  w.bytes = grown;
  *out = w.ptr;
  return TDX_OK;
}

int make_lattice(const double cell[9], Lattice *L) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) L->a[i][j] = cell[3 * i + j];
  const double(*a)[3] = L->a;
  double det = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
               a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
               a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
  if (!(std::fabs(det) > 0) || !std::isfinite(det))
    return fail(TDX_ERR_INVALID_ARG, "cell is singular");
  L->volume = std::fabs(det);
  // b_i = 2 pi (a_j x a_k) / det, cyclic
  for (int i = 0; i < 3; ++i) {
    const double *u = a[(i + 1) % 3], *v = a[(i + 2) % 3];
    double c[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2],
                   u[0] * v[1] - u[1] * v[0]};
    for (int j = 0; j < 3; ++j) L->b[i][j] = 2.0 * M_PI * c[j] / det;
  }
  return TDX_OK;
}

void kq_map(const int N[3], const int qj[3], std::vector<int> *kp, std::vector<int> *gs) {
  const int nk = N[0] * N[1] * N[2];
  kp->resize(nk);
  gs->resize(3 * (size_t)nk);
  for (int k = 0; k < nk; ++k) {
    int r[3];
    kindex_split(k, N, r);
    int rp[3];
    for (int i = 0; i < 3; ++i) {
      int s = r[i] + qj[i];
      int m = ((s % N[i]) + N[i]) % N[i];
      rp[i] = m;
      (*gs)[3 * k + i] = (s - m) / N[i];
    }
    (*kp)[k] = (rp[0] * N[1] + rp[1]) * N[2] + rp[2];
  }
}

static double norm3(const double *v) { return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

void gsphere(const Lattice &L, const double kred[3], double ecut, std::vector<int> *out) {
  double kc[3];
  for (int j = 0; j < 3; ++j)
    kc[j] = kred[0] * L.b[0][j] + kred[1] * L.b[1][j] + kred[2] * L.b[2][j];
  const double kmax = std::sqrt(2.0 * ecut);
  int bound[3];
  for (int i = 0; i < 3; ++i)
    bound[i] = (int)std::floor((kmax + norm3(kc)) * norm3(L.a[i]) / (2.0 * M_PI)) + 1;
  struct E {
    double e;
    int m[3];
  };
  std::vector<E> list;
  for (int x = -bound[0]; x <= bound[0]; ++x)
    for (int y = -bound[1]; y <= bound[1]; ++y)
      for (int z = -bound[2]; z <= bound[2]; ++z) {
        double p[3];
        for (int j = 0; j < 3; ++j)
          p[j] = kc[j] + x * L.b[0][j] + y * L.b[1][j] + z * L.b[2][j];
        double e = 0.5 * (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
        if (e <= ecut) list.push_back({e, {x, y, z}});
      }
  std::sort(list.begin(), list.end(), [](const E &a, const E &b) {
    if (a.e != b.e) return a.e < b.e;
    return std::lexicographical_compare(a.m, a.m + 3, b.m, b.m + 3);
  });
  out->resize(3 * list.size());
  for (size_t i = 0; i < list.size(); ++i)
    for (int j = 0; j < 3; ++j) (*out)[3 * i + j] = list[i].m[j];
}

int check_device(tdx_ctx *ctx) {
  TDX_HIP(hipSetDevice(ctx->device));
  return TDX_OK;
}

}  // namespace tdx

using namespace tdx;

extern "C" {

const char *tdx_last_error(void) { return g_error.c_str(); }

int tdx_abi_version(void) { return TDX_ABI_VERSION; }

int tdx_create(int device, tdx_ctx **out) {
  clear_error();
  TDX_REQUIRE(out, TDX_ERR_INVALID_ARG, "out is null");
  int n = 0;
  TDX_HIP(hipGetDeviceCount(&n));
  TDX_REQUIRE(device >= 0 && device < n, TDX_ERR_INVALID_ARG, "device %d of %d", device, n);
  hipDeviceProp_t prop;
  TDX_HIP(hipGetDeviceProperties(&prop, device));
  TDX_REQUIRE(std::strncmp(prop.gcnArchName, "gfx950", 6) == 0, TDX_ERR_UNSUPPORTED,
              "device %d is %s, this library is built for gfx950", device, prop.gcnArchName);
  TDX_HIP(hipSetDevice(device));
  TDX_TRY(dyson_scratch_init(device));
  tdx_ctx *ctx = new tdx_ctx();
  ctx->device = device;
  ctx->n_cu = prop.multiProcessorCount;
  if (rocblas_create_handle(&ctx->blas) != rocblas_status_success) {
    delete ctx;
    return fail(TDX_ERR_HIP, "rocblas_create_handle failed");
  }
  *out = ctx;
  return TDX_OK;
}

int tdx_destroy(tdx_ctx *ctx) {
  clear_error();
  if (!ctx) return TDX_OK;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  for (auto &w : ctx->ws)
    if (w.ptr) hipFree(w.ptr);
  if (ctx->blas) rocblas_destroy_handle(ctx->blas);
  delete ctx;
  return TDX_OK;
}

int tdx_set_workspace_limit(tdx_ctx *ctx, size_t bytes) {
  clear_error();
  TDX_REQUIRE(ctx, TDX_ERR_INVALID_ARG, "ctx is null");
  ctx->limit = bytes;
  return TDX_OK;
}

int tdx_response_basis(const double cell[9], const int kgrid[3], const int qj[3],
                       double ecut_chi, int *miller_out, int capacity, int *n_out,
                       int *i_g0) {
  clear_error();
  TDX_REQUIRE(cell && kgrid && qj && n_out && i_g0, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(kgrid[0] > 0 && kgrid[1] > 0 && kgrid[2] > 0, TDX_ERR_INVALID_ARG, "bad kgrid");
  TDX_REQUIRE(std::isfinite(ecut_chi) && ecut_chi > 0, TDX_ERR_INVALID_ARG, "bad ecut_chi");
  Lattice L;
  TDX_TRY(make_lattice(cell, &L));
  double qred[3] = {(double)qj[0] / kgrid[0], (double)qj[1] / kgrid[1], (double)qj[2] / kgrid[2]};
  std::vector<int> m;
  gsphere(L, qred, ecut_chi, &m);
  // drop q + G = 0
  std::vector<int> keep;
  int g0 = -1;
  for (size_t i = 0; i < m.size() / 3; ++i) {
    double p[3];
    for (int j = 0; j < 3; ++j)
      p[j] = (qred[0] + m[3 * i]) * L.b[0][j] + (qred[1] + m[3 * i + 1]) * L.b[1][j] +
             (qred[2] + m[3 * i + 2]) * L.b[2][j];
    if (p[0] * p[0] + p[1] * p[1] + p[2] * p[2] <= 1e-20) continue;
    if (m[3 * i] == 0 && m[3 * i + 1] == 0 && m[3 * i + 2] == 0) g0 = (int)keep.size() / 3;
    keep.insert(keep.end(), &m[3 * i], &m[3 * i] + 3);
  }
  const int n = (int)keep.size() / 3;
  *n_out = n;
  *i_g0 = g0;
  TDX_REQUIRE(g0 >= 0, TDX_ERR_INVALID_ARG, "G = 0 (q+G = q) is outside the response basis");
  TDX_REQUIRE(miller_out && capacity >= n, TDX_ERR_SHAPE, "basis has %d vectors, capacity %d",
              n, capacity);
  std::memcpy(miller_out, keep.data(), sizeof(int) * keep.size());
  return TDX_OK;
}

int tdx_momentum(const double cell[9], const int kgrid[3], const int qj[3], double *q_out,
                 double *q2_out) {
  clear_error();
  TDX_REQUIRE(cell && kgrid && qj, TDX_ERR_INVALID_ARG, "null argument");
  TDX_REQUIRE(kgrid[0] > 0 && kgrid[1] > 0 && kgrid[2] > 0, TDX_ERR_INVALID_ARG, "bad kgrid");
  Lattice L;
  TDX_TRY(make_lattice(cell, &L));
  double q[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) q[j] += (double)qj[i] / kgrid[i] * L.b[i][j];
  if (q_out)
    for (int j = 0; j < 3; ++j) q_out[j] = q[j];
  if (q2_out) *q2_out = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
  return TDX_OK;
}

}  // extern "C"
