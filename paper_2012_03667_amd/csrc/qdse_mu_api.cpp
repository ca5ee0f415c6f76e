// qdse_mu_api.cpp -- C ABI of the finite-mu solver (include/qdse.h):
// context set-up, sweeps and the successive-approximation driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "qdse_internal.h"

using namespace qdse;

struct qdse_mu_ctx {
  hipStream_t stream = nullptr;
  HostMuGrid hg;
  int n_inst = 0;
  std::vector<qdse_mu_params> params;
  double *d_ps = nullptr, *d_p4 = nullptr, *d_qs = nullptr, *d_q4 = nullptr, *d_wqs = nullptr,
         *d_wq4 = nullptr, *d_z = nullptr, *d_wz = nullptr, *d_sw_s = nullptr, *d_sw_4 = nullptr;
  int *d_lo_s = nullptr, *d_lo_4 = nullptr;
  double* d_L = nullptr;      // interpolated loop values [inst][3][nl] complex
  double* d_xb[2] = {nullptr, nullptr};
  unsigned long long* d_stat = nullptr;
  MuInst* d_inst = nullptr;        // per-instance constants of the sweep
  int* d_act = nullptr;            // per-instance activity of masked sweeps
  std::vector<int> act_h;          // the mask last uploaded
  unsigned long long* h_stat = nullptr;  // page-locked copy of the statistics
  hipEvent_t ev = nullptr;
};

namespace {

int mu_validate(const qdse_mu_grid* g) {
  if (!g) return QDSE_EINVAL;
  if (g->n_space < 4 || g->n_time < 4 || g->n_space > 4096 || g->n_time > 4096) return QDSE_EINVAL;
  if (g->n_angle < 1 || g->n_angle > 256) return QDSE_EINVAL;
  if (g->interp_order != 1 && g->interp_order != 3) return QDSE_EINVAL;
  if (!(g->r_min > 0.0) || !(g->r_max > g->r_min) || !std::isfinite(g->r_max)) return QDSE_EINVAL;
  if (!(g->T >= 0.0) || !std::isfinite(g->T)) return QDSE_EINVAL;
  if (g->T == 0.0 &&
      (!(g->p4_max > 0.0) || !(g->lam4 > 0.0) || !std::isfinite(g->p4_max)))
    return QDSE_EINVAL;
  return QDSE_OK;
}

template <class T>
int up(T** d, const std::vector<T>& h, hipStream_t st) {
  if (hipMalloc((void**)d, h.size() * sizeof(T)) != hipSuccess) {
    *d = nullptr;
    return QDSE_ENOMEM;
  }
  if (hipMemcpyAsync(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st) != hipSuccess)
    return QDSE_EDEVICE;
  return QDSE_OK;
}

size_t mu_xlen(const qdse_mu_ctx* c) {  // doubles per batch
  return (size_t)c->n_inst * 3 * c->hg.ns * c->hg.n4 * 2;
}

}  // namespace

extern "C" {

int qdse_mu_grid_nodes(const qdse_mu_grid* grid, double* ps, double* p4, double* qs, double* q4,
                       double* wqs, double* wq4, double* z, double* wz) {
  if (mu_validate(grid)) return QDSE_EINVAL;
  HostMuGrid h;
  if (build_mu_grid(*grid, &h)) return QDSE_EINVAL;
  auto put = [](double* d, const std::vector<double>& v) {
    if (d) std::memcpy(d, v.data(), v.size() * sizeof(double));
  };
  put(ps, h.ps);
  put(p4, h.p4);
  put(qs, h.qs);
  put(q4, h.q4);
  put(wqs, h.wqs);
  put(wq4, h.wq4);
  put(z, h.z);
  put(wz, h.wz);
  return QDSE_OK;
}

void qdse_mu_destroy(qdse_mu_ctx* c) {
  if (!c) return;
  void* ptrs[] = {c->d_ps,   c->d_p4,   c->d_qs, c->d_q4,    c->d_wqs,   c->d_wq4, c->d_z,
                  c->d_wz,   c->d_sw_s, c->d_sw_4, c->d_lo_s, c->d_lo_4, c->d_L,   c->d_xb[0],
                  c->d_xb[1], c->d_stat, c->d_inst, c->d_act};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->h_stat) (void)hipHostFree(c->h_stat);
  if (c->ev) (void)hipEventDestroy(c->ev);
  delete c;
}

int qdse_mu_setup(const qdse_mu_grid* grid, const qdse_mu_params* params, int n_inst,
                  void* hip_stream, qdse_mu_ctx** out) {
  if (!out) return QDSE_EINVAL;
  *out = nullptr;
  if (mu_validate(grid) || !params || n_inst < 1 || n_inst > 65535) return QDSE_EINVAL;
  for (int k = 0; k < n_inst; ++k) {
    const qdse_mu_params& p = params[k];
    if (!(p.D >= 0.0) || !std::isfinite(p.D) || !(p.omega > 0.0) || !std::isfinite(p.omega) ||
        !std::isfinite(p.m) || !(p.mu >= 0.0) || !std::isfinite(p.mu))
      return QDSE_EINVAL;
  }
  qdse_mu_ctx* c = new (std::nothrow) qdse_mu_ctx();
  if (!c) return QDSE_ENOMEM;
  c->stream = (hipStream_t)hip_stream;
  c->n_inst = n_inst;
  c->params.assign(params, params + n_inst);
  if (build_mu_grid(*grid, &c->hg)) {
    delete c;
    return QDSE_EINVAL;
  }
  const HostMuGrid& h = c->hg;
  hipStream_t st = c->stream;
  int rc = QDSE_OK;
  if (!rc) rc = up(&c->d_ps, h.ps, st);
  if (!rc) rc = up(&c->d_p4, h.p4, st);
  if (!rc) rc = up(&c->d_qs, h.qs, st);
  if (!rc) rc = up(&c->d_q4, h.q4, st);
  if (!rc) rc = up(&c->d_wqs, h.wqs, st);
  if (!rc) rc = up(&c->d_wq4, h.wq4, st);
  if (!rc) rc = up(&c->d_z, h.z, st);
  if (!rc) rc = up(&c->d_wz, h.wz, st);
  if (!rc) rc = up(&c->d_sw_s, h.sw_s, st);
  if (!rc) rc = up(&c->d_sw_4, h.sw_4, st);
  if (!rc) rc = up(&c->d_lo_s, h.lo_s, st);
  if (!rc) rc = up(&c->d_lo_4, h.lo_4, st);
  const size_t nl = (size_t)h.nqs * h.nq4;
  if (!rc && hipMalloc((void**)&c->d_L, (size_t)n_inst * 3 * nl * 2 * sizeof(double)) != hipSuccess)
    rc = QDSE_ENOMEM;
  for (int b = 0; b < 2 && !rc; ++b)
    if (hipMalloc((void**)&c->d_xb[b], mu_xlen(c) * sizeof(double)) != hipSuccess) rc = QDSE_ENOMEM;
  if (!rc && hipMalloc((void**)&c->d_stat, (size_t)n_inst * sizeof(unsigned long long)) != hipSuccess)
    rc = QDSE_ENOMEM;
  if (!rc) {
    const double pi = 3.14159265358979323846;
    std::vector<MuInst> ih(n_inst);
    for (int k = 0; k < n_inst; ++k) {
      const qdse_mu_params& p = params[k];
      const double o2 = p.omega * p.omega;
      ih[k] = MuInst{p.mu, 8.0 * pi * pi * p.D / (o2 * o2), 1.0 / o2, p.m};
    }
    rc = up(&c->d_inst, ih, st);
  }
  c->act_h.assign(n_inst, 1);
  if (!rc) rc = up(&c->d_act, c->act_h, st);
  if (!rc && hipHostMalloc((void**)&c->h_stat, (size_t)n_inst * sizeof(unsigned long long),
                           hipHostMallocDefault) != hipSuccess) {
    c->h_stat = nullptr;
    rc = QDSE_ENOMEM;
  }
  if (!rc && hipEventCreateWithFlags(&c->ev, hipEventDisableTiming) != hipSuccess) {
    c->ev = nullptr;
    rc = QDSE_EDEVICE;
  }
  if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = QDSE_EDEVICE;
  if (rc) {
    qdse_mu_destroy(c);
    return rc;
  }
  *out = c;
  return QDSE_OK;
}

// One sweep of every instance whose flag in `frozen` is 0 (nullptr: all),
// all instances in one launch with their own mu, interaction and mass;
// frozen instances are copied forward.
static int mu_sweep(qdse_mu_ctx* c, const double* in, double* out, const std::vector<int>* frozen) {
  const HostMuGrid& h = c->hg;
  const int* act = nullptr;
  if (frozen) {
    bool changed = false;
    for (int k = 0; k < c->n_inst; ++k) {
      const int a = (*frozen)[k] ? 0 : 1;
      if (a != c->act_h[k]) changed = true;
      c->act_h[k] = a;
    }
    if (changed && hipMemcpyAsync(c->d_act, c->act_h.data(), c->n_inst * sizeof(int),
                                  hipMemcpyHostToDevice, c->stream) != hipSuccess)
      return QDSE_EDEVICE;
    act = c->d_act;
  }
  hipError_t e = launch_mu_sweep(c->stream, c->n_inst, h.ns, h.n4, h.nqs, h.nq4, h.na, c->d_ps,
                                 c->d_p4, c->d_qs, c->d_q4, c->d_wqs, c->d_wq4, c->d_z, c->d_wz,
                                 c->d_lo_s, c->d_sw_s, c->d_lo_4, c->d_sw_4, c->d_inst, act, in,
                                 out, c->d_L);
  return e == hipSuccess ? QDSE_OK : QDSE_EDEVICE;
}

// Successive approximation of one context as a sequence of steps, so that
// several contexts (grid classes) can run on their own streams together:
// enqueue() puts one sweep of the running instances and its statistic on the
// stream, collect() waits for it and freezes the instances that passed.
struct MuRun {
  qdse_mu_ctx* c = nullptr;
  double* d_x = nullptr;
  double tol = 0.0;
  int max_iter = 0, k = 0, cur = 0, rc = QDSE_OK;
  bool finished = false;
  std::vector<int> done, it;
  std::vector<double> res;

  int begin(qdse_mu_ctx* c_, double* d_x_, double tol_, int max_iter_) {
    c = c_;
    d_x = d_x_;
    tol = tol_;
    max_iter = max_iter_;
    k = 0;
    cur = 0;
    rc = QDSE_OK;
    finished = false;
    done.assign(c->n_inst, 0);
    it.assign(c->n_inst, 0);
    res.assign(c->n_inst, INFINITY);
    if (hipMemcpyAsync(c->d_xb[0], d_x, mu_xlen(c) * sizeof(double), hipMemcpyDeviceToDevice,
                       c->stream) != hipSuccess)
      return QDSE_EDEVICE;
    return QDSE_OK;
  }
  int enqueue() {
    hipStream_t st = c->stream;
    const int ne = c->hg.ns * c->hg.n4;
    ++k;
    if (hipMemsetAsync(c->d_stat, 0, c->n_inst * sizeof(unsigned long long), st) != hipSuccess)
      return QDSE_EDEVICE;
    int r = mu_sweep(c, c->d_xb[cur], c->d_xb[cur ^ 1], &done);
    if (r) return r;
    if (launch_mu_stat(st, c->n_inst, ne, c->d_xb[cur], c->d_xb[cur ^ 1], c->d_stat) != hipSuccess ||
        hipMemcpyAsync(c->h_stat, c->d_stat, c->n_inst * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipEventRecord(c->ev, st) != hipSuccess)
      return QDSE_EDEVICE;
    return QDSE_OK;
  }
  int collect() {
    if (hipEventSynchronize(c->ev) != hipSuccess) return QDSE_EDEVICE;
    cur ^= 1;
    bool all = true, bad = false;
    for (int q = 0; q < c->n_inst; ++q) {
      double r;
      std::memcpy(&r, &c->h_stat[q], sizeof(double));
      if (!done[q]) {
        it[q] = k;
        res[q] = r;
        if (!(r <= 1.7976931348623157e308)) bad = true;
        else if (r < tol) done[q] = 1;  // frozen (copied forward) from the next sweep on
      }
      if (!done[q]) all = false;
    }
    if (all || bad) {
      rc = bad ? QDSE_ENAN : QDSE_OK;
      finished = true;
    } else if (k == max_iter) {
      rc = QDSE_NOT_CONVERGED;
      finished = true;
    }
    return QDSE_OK;
  }
  int end(int* iters, double* resid) {
    if (hipMemcpyAsync(d_x, c->d_xb[cur], mu_xlen(c) * sizeof(double), hipMemcpyDeviceToDevice,
                       c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      return QDSE_EDEVICE;
    for (int q = 0; q < c->n_inst; ++q) {
      if (iters) iters[q] = it[q];
      if (resid) resid[q] = res[q];
    }
    return rc;
  }
};

int qdse_mu_iterate(qdse_mu_ctx* c, const double* d_x_in, double* d_x_out) {
  if (!c || !d_x_in || !d_x_out || d_x_in == d_x_out) return QDSE_EINVAL;
  return mu_sweep(c, d_x_in, d_x_out, nullptr);
}

int qdse_mu_solve(qdse_mu_ctx* c, double* d_x, double tol, int max_iter, int* iters,
                  double* resid) {
  if (!c || !d_x || !(tol > 0.0) || max_iter < 1) return QDSE_EINVAL;
  MuRun r;
  int rc = r.begin(c, d_x, tol, max_iter);
  while (!rc && !r.finished) {
    if ((rc = r.enqueue())) break;
    rc = r.collect();
  }
  if (rc) return rc;
  return r.end(iters, resid);
}

int qdse_mu_solve_group(qdse_mu_ctx** ctxs, int n_ctx, double** d_x, double tol, int max_iter,
                        int** iters, double** resid) {
  if (!ctxs || !d_x || n_ctx < 1 || !(tol > 0.0) || max_iter < 1) return QDSE_EINVAL;
  for (int q = 0; q < n_ctx; ++q) {
    if (!ctxs[q] || !d_x[q]) return QDSE_EINVAL;
    for (int p = 0; p < q; ++p)
      if (ctxs[p] == ctxs[q]) return QDSE_EINVAL;
  }
  std::vector<MuRun> R(n_ctx);
  for (int q = 0; q < n_ctx; ++q)
    if (int rc = R[q].begin(ctxs[q], d_x[q], tol, max_iter)) return rc;
  for (;;) {
    bool any = false;
    for (MuRun& r : R)  // one sweep of every unfinished context, each on its stream
      if (!r.finished) {
        any = true;
        if (int rc = r.enqueue()) return rc;
      }
    if (!any) break;
    for (MuRun& r : R)
      if (!r.finished && r.k > 0)
        if (int rc = r.collect()) return rc;
  }
  int worst = QDSE_OK;
  for (int q = 0; q < n_ctx; ++q) {
    const int rc = R[q].end(iters ? iters[q] : nullptr, resid ? resid[q] : nullptr);
    if (rc < 0 && (worst >= 0 || rc < worst)) worst = rc;
    else if (rc > 0 && worst == QDSE_OK) worst = rc;
  }
  return worst;
}

int qdse_mu_solve_anderson(qdse_mu_ctx* c, double* d_x, double tol, int max_iter, int depth,
                           int* iters, double* resid) {
  if (!c || !d_x || !(tol > 0.0) || max_iter < 1 || depth < 0 || depth > 16) return QDSE_EINVAL;
  hipStream_t st = c->stream;
  const HostMuGrid& h = c->hg;
  const int ne = h.ns * h.n4;
  const size_t L = (size_t)3 * ne * 2;  // doubles per instance (complex as pairs)
  const int nI = c->n_inst, m = depth;
  // per instance: x, g = F(x), f = g - x, previous f and g, and the histories
  // dF[m], dG[m] of their differences (ring buffers)
  std::vector<double*> bufs;
  auto alloc = [&](double** p, size_t n) -> int {
    if (hipMalloc((void**)p, n * sizeof(double)) != hipSuccess) {
      *p = nullptr;
      return QDSE_ENOMEM;
    }
    bufs.push_back(*p);
    return QDSE_OK;
  };
  struct Free {
    std::vector<double*>& b;
    ~Free() {
      for (double* p : b) (void)hipFree(p);
    }
  } guard{bufs};
  double *d_g, *d_f, *d_fp, *d_gp, *d_dF, *d_dG, *d_dot;
  int rc;
  if ((rc = alloc(&d_g, L * nI)) || (rc = alloc(&d_f, L * nI)) || (rc = alloc(&d_fp, L * nI)) ||
      (rc = alloc(&d_gp, L * nI)) || (rc = alloc(&d_dF, L * nI * (m > 0 ? m : 1))) ||
      (rc = alloc(&d_dG, L * nI * (m > 0 ? m : 1))) || (rc = alloc(&d_dot, (size_t)(m + 1) * (m + 1))))
    return rc;
  double* d_xc = c->d_xb[0];
  if (hipMemcpyAsync(d_xc, d_x, mu_xlen(c) * sizeof(double), hipMemcpyDeviceToDevice, st) !=
      hipSuccess)
    return QDSE_EDEVICE;
  std::vector<int> done(nI, 0), it(nI, 0), hist(nI, 0), head(nI, 0);
  std::vector<double> res(nI, INFINITY);
  std::vector<unsigned long long> bits(nI);
  std::vector<double> G((size_t)(m + 1) * (m + 1)), gam(m > 0 ? m : 1);
  rc = QDSE_NOT_CONVERGED;
  for (int k = 1; k <= max_iter; ++k) {
    // g = F(x) for the running instances, statistic max |g - x|
    std::vector<unsigned long long> zero(nI, 0ull);
    if (hipMemcpyAsync(c->d_stat, zero.data(), zero.size() * sizeof(unsigned long long),
                       hipMemcpyHostToDevice, st) != hipSuccess)
      return QDSE_EDEVICE;
    if (int e = mu_sweep(c, d_xc, d_g, &done)) return e;
    if (launch_mu_stat(st, nI, ne, d_xc, d_g, c->d_stat) != hipSuccess) return QDSE_EDEVICE;
    if (hipMemcpyAsync(bits.data(), c->d_stat, nI * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return QDSE_EDEVICE;
    bool all = true, bad = false;
    for (int q = 0; q < nI; ++q) {
      if (done[q]) continue;
      double r;
      std::memcpy(&r, &bits[q], sizeof(double));
      it[q] = k;
      res[q] = r;
      if (!(r <= 1.7976931348623157e308)) bad = true;
      else if (r < tol) done[q] = 2;  // the image g is returned for this instance
      if (!done[q]) all = false;
    }
    if (bad) {
      rc = QDSE_ENAN;
      break;
    }
    for (int q = 0; q < nI; ++q) {
      double* xq = d_xc + q * L;
      double* gq = d_g + q * L;
      if (done[q] == 2) {  // converged on this sweep: keep F(x)
        if (hipMemcpyAsync(xq, gq, L * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
          return QDSE_EDEVICE;
        done[q] = 1;
        continue;
      }
      if (done[q]) continue;
      double* fq = d_f + q * L;
      double* fpq = d_fp + q * L;
      double* gpq = d_gp + q * L;
      double* dFq = d_dF + (size_t)q * m * L;
      double* dGq = d_dG + (size_t)q * m * L;
      if (launch_axpby(st, 1, (int)L, -1.0, xq, nullptr, gq, fq) != hipSuccess)  // f = g - x
        return QDSE_EDEVICE;
      if (m > 0 && k > 1) {  // new history column: f - f_prev, g - g_prev
        const int slot = head[q];
        if (launch_axpby(st, 1, (int)L, -1.0, fpq, nullptr, fq, dFq + slot * L) != hipSuccess ||
            launch_axpby(st, 1, (int)L, -1.0, gpq, nullptr, gq, dGq + slot * L) != hipSuccess)
          return QDSE_EDEVICE;
        head[q] = (slot + 1) % m;
        if (hist[q] < m) ++hist[q];
      }
      if (m > 0 &&
          (hipMemcpyAsync(fpq, fq, L * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess ||
           hipMemcpyAsync(gpq, gq, L * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess))
        return QDSE_EDEVICE;
      const int mk = hist[q];
      if (mk == 0) {  // plain successive approximation step
        if (hipMemcpyAsync(xq, gq, L * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
          return QDSE_EDEVICE;
        continue;
      }
      // least squares min |f - dF gamma|: normal equations dF^T dF gamma = dF^T f
      for (int a = 0; a < mk; ++a)
        if (launch_batched_dot(st, 1, (int)L, dFq, L, dFq + a * L, L, mk,
                               d_dot + (size_t)a * mk) != hipSuccess)
          return QDSE_EDEVICE;
      if (launch_batched_dot(st, 1, (int)L, dFq, L, fq, L, mk, d_dot + (size_t)mk * mk) !=
          hipSuccess)
        return QDSE_EDEVICE;
      if (hipMemcpyAsync(G.data(), d_dot, (size_t)(mk + 1) * mk * sizeof(double),
                         hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return QDSE_EDEVICE;
      // G[a * mk + b] = <dF_b, dF_a>; rhs[b] = G[mk * mk + b]; Tikhonov shift
      // of 1e-14 of the largest diagonal keeps nearly dependent columns solvable
      std::vector<double> Aq((size_t)mk * mk), bq(mk);
      double dmax = 0.0;
      for (int a = 0; a < mk; ++a) dmax = std::fmax(dmax, G[(size_t)a * mk + a]);
      for (int a = 0; a < mk; ++a) {
        for (int b = 0; b < mk; ++b) Aq[(size_t)a * mk + b] = G[(size_t)a * mk + b];
        Aq[(size_t)a * mk + a] += 1e-14 * dmax;
        bq[a] = G[(size_t)mk * mk + a];
      }
      for (int a = 0; a < mk; ++a) {  // Gaussian elimination with partial pivoting
        int piv = a;
        for (int r = a + 1; r < mk; ++r)
          if (std::fabs(Aq[(size_t)r * mk + a]) > std::fabs(Aq[(size_t)piv * mk + a])) piv = r;
        if (piv != a) {
          for (int b = 0; b < mk; ++b) std::swap(Aq[(size_t)a * mk + b], Aq[(size_t)piv * mk + b]);
          std::swap(bq[a], bq[piv]);
        }
        const double d = Aq[(size_t)a * mk + a];
        if (d == 0.0) continue;
        for (int r = a + 1; r < mk; ++r) {
          const double f = Aq[(size_t)r * mk + a] / d;
          for (int b = a; b < mk; ++b) Aq[(size_t)r * mk + b] -= f * Aq[(size_t)a * mk + b];
          bq[r] -= f * bq[a];
        }
      }
      for (int a = mk - 1; a >= 0; --a) {
        double acc = bq[a];
        for (int b = a + 1; b < mk; ++b) acc -= Aq[(size_t)a * mk + b] * gam[b];
        const double d = Aq[(size_t)a * mk + a];
        gam[a] = d != 0.0 ? acc / d : 0.0;
      }
      // x = g - dG gamma
      for (int a = 0; a < mk; ++a) gam[a] = -gam[a];
      if (hipMemcpyAsync(xq, gq, L * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess ||
          hipMemcpyAsync(d_dot, gam.data(), mk * sizeof(double), hipMemcpyHostToDevice, st) !=
              hipSuccess ||
          launch_combine(st, 1, (int)L, dGq, L, mk, d_dot, mk, 1.0, xq) != hipSuccess)
        return QDSE_EDEVICE;
    }
    if (all) {
      rc = QDSE_OK;
      break;
    }
  }
  if (hipMemcpyAsync(d_x, d_xc, mu_xlen(c) * sizeof(double), hipMemcpyDeviceToDevice, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return QDSE_EDEVICE;
  for (int q = 0; q < nI; ++q) {
    if (iters) iters[q] = it[q];
    if (resid) resid[q] = res[q];
  }
  return rc;
}

}  // extern "C"
