// qdse_fred_api.cpp -- C ABI of the general second-kind system of Sec. I
// (eqs. jifen1, jifen3, jifen12); see include/qdse.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "qdse_internal.h"

using namespace qdse;

namespace {

constexpr int kChunk = 8;  // sweeps between convergence checks

template <class T>
int falloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return QDSE_OK;
  return hipMalloc((void**)p, count * sizeof(T)) == hipSuccess ? QDSE_OK : QDSE_ENOMEM;
}

bool grid_ok(const qdse_fred_grid* g) {
  return g && g->n >= 4 && g->n <= (1 << 16) && (g->interp_order == 1 || g->interp_order == 3) &&
         std::isfinite(g->a) && std::isfinite(g->b) && g->a < g->b && g->alpha > 0.0 &&
         g->alpha <= 1.0;
}

}  // namespace

namespace qdse {

void gl_nodes_on(int n, double a, double b, double* x, double* w) { gl_mapped(n, a, b, x, w); }

}  // namespace qdse

struct qdse_fred_ctx {
  int n = 0, order = 3;
  double alpha = 0.5;
  hipStream_t stream = nullptr;
  const double *K1 = nullptr, *K2 = nullptr, *f = nullptr;  // the caller's
  double *d_x = nullptr, *d_t = nullptr, *d_w = nullptr, *d_sw = nullptr, *d_coef = nullptr;
  double *d_G = nullptr, *d_ring = nullptr;  // ring: kChunk + 1 iterates
  int* d_lo = nullptr;
  unsigned long long* d_stat = nullptr;
  unsigned long long* h_stat = nullptr;  // pinned
};

extern "C" {

int qdse_fred_nodes(const qdse_fred_grid* grid, double* x, double* t, double* w) {
  if (!grid_ok(grid) || !x || !t || !w) return QDSE_EINVAL;
  std::vector<double> wx(grid->n);
  gl_nodes_on(grid->n, grid->a, grid->b, x, wx.data());
  gl_nodes_on(grid->n + 1, grid->a, grid->b, t, w);
  return QDSE_OK;
}

void qdse_fred_destroy(qdse_fred_ctx* c) {
  if (!c) return;
  void* ptrs[] = {c->d_x, c->d_t, c->d_w, c->d_sw, c->d_coef, c->d_G, c->d_ring, c->d_lo,
                  c->d_stat};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->h_stat) (void)hipHostFree(c->h_stat);
  delete c;
}

int qdse_fred_setup(const qdse_fred_grid* grid, const qdse_fred_poly* F, const double* d_K1,
                    const double* d_K2, const double* d_f, void* hip_stream,
                    qdse_fred_ctx** out) {
  if (!out) return QDSE_EINVAL;
  *out = nullptr;
  if (!grid_ok(grid) || !F || !d_K1 || !d_K2 || !d_f) return QDSE_EINVAL;
  for (int k = 0; k < 4; ++k)
    for (int q = 0; q < 6; ++q)
      if (!std::isfinite(F[k].c[q])) return QDSE_EINVAL;
  qdse_fred_ctx* c = new (std::nothrow) qdse_fred_ctx();
  if (!c) return QDSE_ENOMEM;
  const int n = grid->n, nq = n + 1;
  c->n = n;
  c->order = grid->interp_order;
  c->alpha = grid->alpha;
  c->stream = (hipStream_t)hip_stream;
  c->K1 = d_K1;
  c->K2 = d_K2;
  c->f = d_f;
  std::vector<double> x(n), wx(n), t(nq), w(nq), sw(4 * nq), coef(24);
  std::vector<int> lo(nq);
  gl_nodes_on(n, grid->a, grid->b, x.data(), wx.data());
  gl_nodes_on(nq, grid->a, grid->b, t.data(), w.data());
  build_stencils(n, c->order, x.data(), t.data(), lo.data(), sw.data());
  for (int k = 0; k < 4; ++k) std::memcpy(&coef[6 * k], F[k].c, 6 * sizeof(double));
  int rc = QDSE_OK;
  if (!rc) rc = falloc(&c->d_x, n);
  if (!rc) rc = falloc(&c->d_t, nq);
  if (!rc) rc = falloc(&c->d_w, nq);
  if (!rc) rc = falloc(&c->d_sw, 4 * nq);
  if (!rc) rc = falloc(&c->d_coef, 24);
  if (!rc) rc = falloc(&c->d_G, 4 * (size_t)nq);
  if (!rc) rc = falloc(&c->d_ring, (size_t)(kChunk + 1) * 2 * n);
  if (!rc) rc = falloc(&c->d_lo, nq);
  if (!rc) rc = falloc(&c->d_stat, kChunk);
  if (!rc && hipHostMalloc((void**)&c->h_stat, kChunk * sizeof(unsigned long long),
                           hipHostMallocDefault) != hipSuccess) {
    c->h_stat = nullptr;
    rc = QDSE_ENOMEM;
  }
  hipStream_t st = c->stream;
  auto up = [&](void* d, const void* h, size_t bytes) {
    if (!rc && hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st) != hipSuccess)
      rc = QDSE_EDEVICE;
  };
  up(c->d_x, x.data(), n * sizeof(double));
  up(c->d_t, t.data(), nq * sizeof(double));
  up(c->d_w, w.data(), nq * sizeof(double));
  up(c->d_sw, sw.data(), sw.size() * sizeof(double));
  up(c->d_coef, coef.data(), coef.size() * sizeof(double));
  up(c->d_lo, lo.data(), nq * sizeof(int));
  if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = QDSE_EDEVICE;
  if (rc) {
    qdse_fred_destroy(c);
    return rc;
  }
  *out = c;
  return QDSE_OK;
}

int qdse_fred_iterate(qdse_fred_ctx* c, const double* d_in, double* d_out) {
  if (!c || !d_in || !d_out || d_in == d_out) return QDSE_EINVAL;
  if (launch_fred_sweep(c->stream, c->n, c->alpha, c->d_x, c->d_t, c->d_w, c->d_lo, c->d_sw,
                        c->d_coef, c->K1, c->K2, c->f, d_in, d_out, c->d_G,
                        nullptr) != hipSuccess)
    return QDSE_EDEVICE;
  return QDSE_OK;
}

int qdse_fred_solve(qdse_fred_ctx* c, double* d_uv, double tol, int max_iter, int* iters,
                    double* resid) {
  if (!c || !d_uv || !(tol > 0.0) || max_iter < 1) return QDSE_EINVAL;
  hipStream_t st = c->stream;
  const size_t len = 2 * (size_t)c->n;
  auto buf = [&](long k) { return c->d_ring + (size_t)(k % (kChunk + 1)) * len; };
  if (hipMemcpyAsync(buf(0), d_uv, len * sizeof(double), hipMemcpyDeviceToDevice, st) !=
      hipSuccess)
    return QDSE_EDEVICE;
  long done = 0, hit = -1;
  double r = INFINITY;
  int rc = QDSE_NOT_CONVERGED;
  while (done < max_iter && hit < 0) {
    const int m = (int)std::min<long>(kChunk, max_iter - done);
    if (hipMemsetAsync(c->d_stat, 0, m * sizeof(unsigned long long), st) != hipSuccess)
      return QDSE_EDEVICE;
    for (int q = 0; q < m; ++q)
      if (launch_fred_sweep(st, c->n, c->alpha, c->d_x, c->d_t, c->d_w, c->d_lo, c->d_sw,
                            c->d_coef, c->K1, c->K2, c->f, buf(done + q), buf(done + q + 1),
                            c->d_G, c->d_stat + q) != hipSuccess)
        return QDSE_EDEVICE;
    if (hipMemcpyAsync(c->h_stat, c->d_stat, m * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return QDSE_EDEVICE;
    for (int q = 0; q < m && hit < 0; ++q) {
      std::memcpy(&r, &c->h_stat[q], sizeof(double));
      if (!(r <= 1.7976931348623157e308)) {
        hit = done + q + 1;
        rc = QDSE_ENAN;
      } else if (r < tol) {
        hit = done + q + 1;
        rc = QDSE_OK;
      }
    }
    done += m;
  }
  const long last = hit > 0 ? hit : done;
  if (hipMemcpyAsync(d_uv, buf(last), len * sizeof(double), hipMemcpyDeviceToDevice, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return QDSE_EDEVICE;
  if (iters) *iters = (int)last;
  if (resid) *resid = r;
  return rc;
}

int qdse_fred_time_sweep(qdse_fred_ctx* c, const double* d_in, double* d_out, int reps,
                         double* avg_ms) {
  if (!c || !d_in || !d_out || d_in == d_out || reps < 1 || !avg_ms) return QDSE_EINVAL;
  std::vector<hipEvent_t> ev(2 * reps, nullptr);
  int rc = QDSE_OK;
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) rc = QDSE_EDEVICE;
  for (int r = 0; r < reps && rc == QDSE_OK; ++r)
    if (launch_fred_sweep(c->stream, c->n, c->alpha, c->d_x, c->d_t, c->d_w, c->d_lo, c->d_sw,
                          c->d_coef, c->K1, c->K2, c->f, d_in, d_out, c->d_G, c->d_stat,
                          ev[2 * r], ev[2 * r + 1]) != hipSuccess)
      rc = QDSE_EDEVICE;
  double tot = 0.0;
  if (rc == QDSE_OK && hipStreamSynchronize(c->stream) == hipSuccess) {
    for (int r = 0; r < reps; ++r) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]) != hipSuccess) rc = QDSE_EDEVICE;
      tot += ms;
    }
  } else if (rc == QDSE_OK) {
    rc = QDSE_EDEVICE;
  }
  for (auto e : ev)
    if (e) (void)hipEventDestroy(e);
  if (rc == QDSE_OK) *avg_ms = tot / reps;
  return rc;
}

}  // extern "C"
