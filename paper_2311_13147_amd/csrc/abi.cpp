// C ABI of libcsot (declared in include/csot.h): argument validation, error reporting,
// workspace sizing and dispatch to the kernel launchers.  Validation runs on the host before
// any HIP call, so invalid arguments are rejected without touching a device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "csot.h"
#include "launch.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int ok() {
  g_last_error.clear();
  return OT_OK;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(OT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

ot_opts defaults() {
  ot_opts o;
  std::memset(&o, 0, sizeof(o));
  o.tol = 1e-6;
  o.max_iter = 10000;
  o.fold_fp64 = -1;
  return o;
}

int check_problem(const ot_problem* p, bool need_points_or_cost = true) {
  if (!p) return fail(OT_ERR_ARG, "problem is NULL");
  if (p->n <= 0) return fail(OT_ERR_ARG, "n must be positive (got %d)", p->n);
  if (p->K <= 0) return fail(OT_ERR_ARG, "K must be positive (got %d)", p->K);
  if (p->n % p->K != 0) return fail(OT_ERR_ARG, "n (%d) is not a multiple of K (%d)", p->n, p->K);
  if (!(p->eps > 0.0) || !std::isfinite(p->eps))
    return fail(OT_ERR_ARG, "eps must be positive and finite");
  if (!p->a || !p->b) return fail(OT_ERR_ARG, "marginals a and b must be non-NULL");
  if (need_points_or_cost) {
    if (p->dim == 2 || p->dim == 3) {
      if (!p->x || !p->y) return fail(OT_ERR_ARG, "dim=%d needs coordinates x and y", p->dim);
    } else if (p->dim == 0) {
      if (!p->C) return fail(OT_ERR_ARG, "dim=0 needs a dense cost C");
      if (p->ldc < p->n) return fail(OT_ERR_ARG, "ldc (%lld) < n (%d)", (long long)p->ldc, p->n);
    } else {
      return fail(OT_ERR_ARG, "dim must be 0, 2 or 3 (got %d)", p->dim);
    }
  }
  return OT_OK;
}

int check_opts(const ot_opts& o) {
  if (!(o.tol >= 0.0) || !std::isfinite(o.tol)) return fail(OT_ERR_ARG, "tol must be >= 0");
  if (o.max_iter < 1) return fail(OT_ERR_ARG, "max_iter must be >= 1");
  if (o.fold_fp64 < -1 || o.fold_fp64 > 1) return fail(OT_ERR_ARG, "fold_fp64 must be -1, 0 or 1");
  if (o.workgroups < 0) return fail(OT_ERR_ARG, "workgroups must be >= 0");
  if (o.warm_start < 0 || o.warm_start > 2) return fail(OT_ERR_ARG, "warm_start must be 0, 1 or 2");
  if (o.reserved != 0) return fail(OT_ERR_ARG, "reserved option field must be 0");
  return OT_OK;
}

int check_ws(const void* ws, size_t have, size_t need) {
  if (need == 0) return OT_OK;
  if (!ws) return fail(OT_ERR_WORKSPACE, "workspace is NULL (need %zu bytes)", need);
  if (have < need) return fail(OT_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", have, need);
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(OT_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  return OT_OK;
}

csot::Geom geom(const ot_problem* p) {
  csot::Geom g;
  g.n = p->n;
  g.K = p->K;
  g.m = p->n / p->K;
  g.dim = p->dim;
  g.x = p->x;
  g.y = p->y;
  g.C = p->C;
  g.ldc = p->ldc;
  g.a = p->a;
  g.b = p->b;
  g.eps = p->eps;
  return g;
}

// Host-side validation of marginals and (optionally) block-circulance.  Synchronises.
int validate_inputs(const ot_problem* p, hipStream_t s, bool check_symmetry) {
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  std::vector<float> a(p->n), b(p->n);
  if ((e = hipMemcpy(a.data(), p->a, sizeof(float) * p->n, hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "hipMemcpy(a)");
  if ((e = hipMemcpy(b.data(), p->b, sizeof(float) * p->n, hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "hipMemcpy(b)");
  double sa = 0.0, sb = 0.0;
  for (int i = 0; i < p->n; ++i) {
    if (!(a[i] > 0.0f) || !std::isfinite(a[i]))
      return fail(OT_ERR_MASS, "a[%d] = %g is not positive and finite", i, (double)a[i]);
    if (!(b[i] > 0.0f) || !std::isfinite(b[i]))
      return fail(OT_ERR_MASS, "b[%d] = %g is not positive and finite", i, (double)b[i]);
    sa += a[i];
    sb += b[i];
  }
  if (std::fabs(sa - sb) > 1e-6)
    return fail(OT_ERR_MASS, "sum(a) = %.9g differs from sum(b) = %.9g", sa, sb);
  if (!check_symmetry || p->K == 1) return OT_OK;
  const int n = p->n, K = p->K, m = n / K;
  // sample entries C[r m + i, c m + j] and compare with block-row 0's C[i, ((c - r) mod K) m + j]
  auto cost_at = [&](const std::vector<float>& xs, const std::vector<float>& ys, int I, int J) {
    double c = 0.0;
    for (int d = 0; d < p->dim; ++d) {
      const double df = (double)xs[(size_t)I * p->dim + d] - (double)ys[(size_t)J * p->dim + d];
      c += df * df;
    }
    return c;
  };
  unsigned state = 12345u;
  auto rnd = [&](int mod) {
    state = state * 1664525u + 1013904223u;
    return (int)((state >> 8) % (unsigned)mod);
  };
  if (p->dim > 0) {
    std::vector<float> xs((size_t)n * p->dim), ys((size_t)n * p->dim);
    if ((e = hipMemcpy(xs.data(), p->x, sizeof(float) * xs.size(), hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail(e, "hipMemcpy(x)");
    if ((e = hipMemcpy(ys.data(), p->y, sizeof(float) * ys.size(), hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail(e, "hipMemcpy(y)");
    double scale = 0.0;
    for (int s = 0; s < 64; ++s) scale = std::fmax(scale, cost_at(xs, ys, rnd(n), rnd(n)));
    for (int s = 0; s < 256; ++s) {
      const int r = rnd(K), c = rnd(K), i = rnd(m), j = rnd(m);
      const double full = cost_at(xs, ys, r * m + i, c * m + j);
      const double row0 = cost_at(xs, ys, i, ((c - r + K) % K) * m + j);
      if (std::fabs(full - row0) > 1e-5 * (scale + 1e-30))
        return fail(OT_ERR_NOT_SYMMETRIC,
                    "cost entry (%d, %d) = %.9g differs from block-row 0 entry %.9g", r * m + i,
                    c * m + j, full, row0);
    }
  } else {
    for (int s = 0; s < 256; ++s) {
      const int r = rnd(K), c = rnd(K), i = rnd(m), j = rnd(m);
      float v1 = 0.f, v2 = 0.f;
      if ((e = hipMemcpy(&v1, p->C + (int64_t)(r * m + i) * p->ldc + c * m + j, 4, hipMemcpyDeviceToHost)) != hipSuccess ||
          (e = hipMemcpy(&v2, p->C + (int64_t)i * p->ldc + ((c - r + K) % K) * m + j, 4, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "hipMemcpy(C)");
      if (v1 != v2)
        return fail(OT_ERR_NOT_SYMMETRIC, "dense cost is not block-circulant at (%d, %d)",
                    r * m + i, c * m + j);
    }
  }
  return OT_OK;
}

// Copy device statistics into the host struct (synchronises) and map them to a return code.
int finish_stats(const double* dstats, ot_stats* hs, double tol, hipStream_t s) {
  double v[OT_DSTATS_LEN];
  hipError_t e = hipMemcpyAsync(v, dstats, sizeof(v), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "reading solver statistics");
  hs->iters = (int32_t)v[0];
  hs->converged = (int32_t)v[1];
  hs->err_row = v[2];
  hs->err_col = v[3];
  hs->err_row32 = v[4];
  hs->flags = (int32_t)v[5];
  hs->reserved = 0;
  if (hs->flags & 2) return fail(OT_ERR_HIP, "a device-wide barrier timed out");
  if (hs->flags & 1) return fail(OT_ERR_NONFINITE, "a potential became non-finite");
  if (tol > 0.0 && !hs->converged) return fail(OT_ERR_NOCONV, "max_iter reached (err_row32 = %.3e)", hs->err_row32);
  return ok();
}

}  // namespace

extern "C" {

const char* ot_last_error(void) { return g_last_error.c_str(); }

const char* ot_version(void) { return "csot 0.1 (gfx950)"; }

size_t ot_workspace_bytes(const ot_problem* prob, const ot_opts* opts) {
  if (check_problem(prob, false) != OT_OK) return 0;
  ot_opts o = opts ? *opts : defaults();
  const csot::Geom g = geom(prob);
  size_t need = 256;
  // reduced solver: sized for the largest workgroup count it may use (one per CU, <= m)
  {
    csot::ReducedPlan rp;
    rp.W = g.m < 1024 ? g.m : 1024;
    if (o.workgroups > rp.W) rp.W = o.workgroups;
    rp.R = 1;
    rp.stride = 1;
    rp.threads = 256;
    rp.lds = 0;
    // padded logK copies of the large-m mode: needed above m = 2048 on 256 CUs; sized in from
    // m = 1024 so that devices down to 64 CUs are covered
    // a workgroup hint above the CU count also moves the slabs to device memory
    rp.gslab = (g.m > 1024 || o.workgroups > 0) ? 1 : 0;
    need = std::max(need, csot::reduced_ws_bytes(g.m, rp));
    // and whatever the planner decides on the current device (when there is one)
    csot::ReducedPlan actual;
    if (csot::plan_reduced(g.m, o.workgroups, &actual))
      need = std::max(need, csot::reduced_ws_bytes(g.m, actual));
  }
  {
    csot::FullPlan fp;
    fp.W = g.n;
    fp.R = 1;
    fp.P = 1;
    fp.threads = 256;
    fp.lds = 0;
    if (g.dim == 2 || g.dim == 3 || g.dim == 0) need = std::max(need, csot::full_ws_bytes(g, fp));
  }
  need = std::max(need, csot::costgrad_ws_bytes(g));
  return need;
}

int ot_fold_kernel(const ot_problem* prob, const ot_opts* opts, float* logK, float* alpha,
                   float* beta, void* ws, size_t ws_bytes, void* stream) {
  (void)ws;
  (void)ws_bytes;
  int rc = check_problem(prob);
  if (rc) return rc;
  ot_opts o = opts ? *opts : defaults();
  if ((rc = check_opts(o))) return rc;
  if (!logK || !alpha || !beta) return fail(OT_ERR_ARG, "fold outputs must be non-NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (o.validate && (rc = validate_inputs(prob, s, true))) return rc;
  const bool fp64 = o.fold_fp64 != 0;
  hipError_t e = csot::launch_fold(geom(prob), fp64, logK, alpha, beta, s);
  if (e != hipSuccess) return hip_fail(e, "fold launch");
  return ok();
}

int ot_symmetrize_cost(const ot_problem* prob, float* Csym, int64_t ldcs, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!Csym) return fail(OT_ERR_ARG, "Csym must be non-NULL");
  if (ldcs < prob->n) return fail(OT_ERR_ARG, "ldcs (%lld) < n (%d)", (long long)ldcs, prob->n);
  hipError_t e = csot::launch_symmetrize(geom(prob), Csym, ldcs, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "symmetrize launch");
  return ok();
}

int ot_sinkhorn_reduced(const ot_problem* prob, const ot_opts* opts, const float* logK,
                        const float* alpha, const float* beta, float* f, float* g,
                        double* dstats, ot_stats* hstats, void* ws, size_t ws_bytes,
                        void* stream) {
  int rc = check_problem(prob, false);
  if (rc) return rc;
  ot_opts o = opts ? *opts : defaults();
  if ((rc = check_opts(o))) return rc;
  if (!logK || !alpha || !beta || !f || !g)
    return fail(OT_ERR_ARG, "logK, alpha, beta, f and g must be non-NULL");
  if (hstats && !dstats) return fail(OT_ERR_ARG, "host statistics need a device dstats buffer");
  if (!dstats) return fail(OT_ERR_ARG, "dstats must be non-NULL");
  const int m = prob->n / prob->K;
  csot::ReducedPlan plan;
  if (!csot::plan_reduced(m, o.workgroups, &plan))
    return fail(OT_ERR_UNSUPPORTED, "no co-resident launch configuration for m = %d", m);
  if ((rc = check_ws(ws, ws_bytes, csot::reduced_ws_bytes(m, plan)))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = csot::launch_sinkhorn_reduced(m, prob->K, prob->eps, logK, alpha, beta, f, g,
                                               o.tol, o.max_iter, o.warm_start, dstats, ws, plan, s,
                                               static_cast<hipEvent_t*>(o.timing_events));
  if (e != hipSuccess) return hip_fail(e, "reduced solver launch");
  if (hstats) return finish_stats(dstats, hstats, o.tol, s);
  return ok();
}

int ot_sinkhorn_reduced_noalloc(const ot_problem* prob, const ot_opts* opts, const float* logK,
                                const float* alpha, const float* beta, float* f, float* g,
                                double* dstats, ot_stats* hstats, void* stream) {
  int rc = check_problem(prob, false);
  if (rc) return rc;
  ot_opts o = opts ? *opts : defaults();
  if ((rc = check_opts(o))) return rc;
  if (!logK || !alpha || !beta || !f || !g)
    return fail(OT_ERR_ARG, "logK, alpha, beta, f and g must be non-NULL");
  if (!dstats) return fail(OT_ERR_ARG, "dstats must be non-NULL");
  const int m = prob->n / prob->K;
  csot::ReducedPlan plan;
  if (!csot::plan_reduced(m, o.workgroups, &plan))
    return fail(OT_ERR_UNSUPPORTED, "no co-resident launch configuration for m = %d", m);
  const size_t need = csot::reduced_ws_bytes(m, plan);
  if (need > csot::kReducedScratchBytes)
    return fail(OT_ERR_UNSUPPORTED,
                "m = %d needs %zu bytes of scratch%s; the allocation-free call holds %zu", m, need,
                plan.gslab ? " (logK slabs in device memory)" : "", csot::kReducedScratchBytes);
  void* scratch = nullptr;
  hipError_t e = csot::reduced_scratch(&scratch);
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  e = csot::launch_sinkhorn_reduced(m, prob->K, prob->eps, logK, alpha, beta, f, g, o.tol,
                                    o.max_iter, o.warm_start, dstats, scratch, plan, s,
                                    static_cast<hipEvent_t*>(o.timing_events));
  if (e != hipSuccess) return hip_fail(e, "reduced solver launch");
  if (hstats) return finish_stats(dstats, hstats, o.tol, s);
  return ok();
}

int ot_sinkhorn_full(const ot_problem* prob, const ot_opts* opts, float* f, float* g,
                     double* dstats, ot_stats* hstats, void* ws, size_t ws_bytes,
                     void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  ot_opts o = opts ? *opts : defaults();
  if ((rc = check_opts(o))) return rc;
  if (!f || !g) return fail(OT_ERR_ARG, "f and g must be non-NULL");
  if (!dstats) return fail(OT_ERR_ARG, "dstats must be non-NULL");
  const csot::Geom geo = geom(prob);
  csot::FullPlan plan;
  if (!csot::plan_full(geo, o.workgroups, &plan))
    return fail(OT_ERR_UNSUPPORTED, "no co-resident launch configuration for n = %d", prob->n);
  if ((rc = check_ws(ws, ws_bytes, csot::full_ws_bytes(geo, plan)))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (o.validate && (rc = validate_inputs(prob, s, false))) return rc;
  hipError_t e = csot::launch_sinkhorn_full(geo, f, g, o.tol, o.max_iter, o.warm_start, dstats,
                                            ws, plan, s, static_cast<hipEvent_t*>(o.timing_events));
  if (e != hipSuccess) return hip_fail(e, "full solver launch");
  if (hstats) return finish_stats(dstats, hstats, o.tol, s);
  return ok();
}

int ot_full_plan_info(const ot_problem* prob, const ot_opts* opts, int32_t* info) {
  int rc = check_problem(prob);
  if (rc) return rc;
  ot_opts o = opts ? *opts : defaults();
  if ((rc = check_opts(o))) return rc;
  if (!info) return fail(OT_ERR_ARG, "info must be non-NULL");
  csot::FullPlan plan;
  if (!csot::plan_full(geom(prob), o.workgroups, &plan))
    return fail(OT_ERR_UNSUPPORTED, "no co-resident launch configuration for n = %d", prob->n);
  info[0] = plan.W;
  info[1] = plan.R;
  info[2] = plan.P;
  info[3] = plan.threads / 100;
  info[4] = plan.threads % 100;
  info[5] = prob->dim == 0 ? 1 : 0;
  return ok();
}

int ot_reduced_plan_info(const ot_problem* prob, const ot_opts* opts, int32_t* info) {
  int rc = check_problem(prob, false);
  if (rc) return rc;
  ot_opts o = opts ? *opts : defaults();
  if ((rc = check_opts(o))) return rc;
  if (!info) return fail(OT_ERR_ARG, "info must be non-NULL");
  csot::ReducedPlan plan;
  const int m = prob->n / prob->K;
  if (!csot::plan_reduced(m, o.workgroups, &plan))
    return fail(OT_ERR_UNSUPPORTED, "no co-resident launch configuration for m = %d", m);
  info[0] = plan.W;
  info[1] = plan.R;
  info[2] = plan.stride;
  info[3] = plan.gslab;
  info[4] = (int32_t)plan.lds;
  info[5] = plan.threads;
  return ok();
}

int ot_expand_plan(const ot_problem* prob, const float* f, const float* g, float* T,
                   int64_t ldt, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!f || !g || !T) return fail(OT_ERR_ARG, "f, g and T must be non-NULL");
  if (ldt < prob->n) return fail(OT_ERR_ARG, "ldt (%lld) < n (%d)", (long long)ldt, prob->n);
  hipError_t e = csot::launch_expand(geom(prob), f, g, T, ldt, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "expand launch");
  return ok();
}

int ot_lot_fold(const ot_problem* prob, float* G, int32_t* kmin, float* alpha, float* beta,
                void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!G || !kmin || !alpha || !beta)
    return fail(OT_ERR_ARG, "G, kmin, alpha and beta must be non-NULL");
  hipError_t e = csot::launch_lot_fold(geom(prob), G, kmin, alpha, beta,
                                       static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "lot fold launch");
  return ok();
}

int ot_lot_expand(const ot_problem* prob, const float* S, const int32_t* kmin, float* T,
                  int64_t ldt, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!S || !kmin || !T) return fail(OT_ERR_ARG, "S, kmin and T must be non-NULL");
  if (ldt < prob->n) return fail(OT_ERR_ARG, "ldt (%lld) < n (%d)", (long long)ldt, prob->n);
  hipError_t e = csot::launch_lot_expand(prob->n / prob->K, prob->K, S, kmin, T, ldt,
                                         static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "lot expand launch");
  return ok();
}

size_t ot_srot_workspace_bytes(const ot_problem* prob) {
  if (!prob || prob->n <= 0 || prob->K <= 0 || prob->n % prob->K) return 0;
  return csot::srot_ws_bytes(geom(prob));
}

int ot_srot_reduced(const ot_problem* prob, double lam, const ot_opts* opts, float* w, float* z,
                    ot_stats* hstats, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  ot_opts o = opts ? *opts : defaults();
  if ((rc = check_opts(o))) return rc;
  if (!(lam > 0.0) || !std::isfinite(lam)) return fail(OT_ERR_ARG, "lam must be > 0");
  if (!w || !z || !hstats) return fail(OT_ERR_ARG, "w, z and hstats must be non-NULL");
  if (o.warm_start == 2) return fail(OT_ERR_ARG, "warm_start must be 0 or 1");
  const csot::Geom geo = geom(prob);
  if ((rc = check_ws(ws, ws_bytes, csot::srot_ws_bytes(geo)))) return rc;
  if (!csot::srot_supported(geo))
    return fail(OT_ERR_UNSUPPORTED, "m = %d: the staged potential exceeds the LDS of a workgroup",
                geo.m);
  double res[6] = {0, 0, 0, 0, 0, 0};
  hipError_t e = csot::run_srot(geo, lam, o.tol, o.max_iter, o.warm_start, w, z, ws, res,
                                static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "srot launch");
  *hstats = ot_stats{};
  hstats->iters = (int32_t)res[0];
  hstats->converged = (int32_t)res[1];
  hstats->err_row = res[2];
  hstats->err_col = res[3];
  hstats->err_row32 = res[2];
  hstats->flags = (int32_t)res[5];
  if ((int32_t)res[5] & 2) return fail(OT_ERR_HIP, "srot solver: an exchange wait timed out");
  if (!std::isfinite(res[2]) || !std::isfinite(res[3]) || ((int32_t)res[5] & 1)) {
    hstats->flags |= 1;
    return fail(OT_ERR_NONFINITE, "non-finite residual");
  }
  if (!hstats->converged && o.tol > 0.0) return fail(OT_ERR_NOCONV, "max_iter reached");
  return ok();
}

int ot_cost_and_grad(const ot_problem* prob, const float* f, const float* g, int32_t reduced,
                     double* out, float* dC, int64_t lddc, float* dx, float* dy, float* da,
                     float* db, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!f || !g || !out) return fail(OT_ERR_ARG, "f, g and out must be non-NULL");
  if (reduced != 0 && reduced != 1) return fail(OT_ERR_ARG, "reduced must be 0 or 1");
  if (prob->dim == 0 && (dx || dy)) return fail(OT_ERR_ARG, "dx/dy need coordinates (dim 2 or 3)");
  if (dC && lddc < prob->n)
    return fail(OT_ERR_ARG, "lddc (%lld) < n (%d)", (long long)lddc, prob->n);
  const csot::Geom geo = geom(prob);
  if ((rc = check_ws(ws, ws_bytes, csot::costgrad_ws_bytes(geo)))) return rc;
  hipError_t e = csot::launch_cost_and_grad(geo, f, g, reduced, out, dC, lddc, dx, dy, da, db,
                                            ws, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "cost_and_grad launch");
  return ok();
}

size_t ot_batched_plan_len(int32_t count) {
  return count > 0 ? csot::batched_plan_len(count) : 0;
}

int ot_batched_plan(const ot_batch_desc* h, int32_t count, int32_t* plan) {
  if (!h || !plan || count <= 0) return fail(OT_ERR_ARG, "descriptors, plan and count > 0 required");
  for (int p = 0; p < count; ++p) {
    const ot_batch_desc& d = h[p];
    if (d.n <= 0 || d.K <= 0 || d.n % d.K != 0)
      return fail(OT_ERR_ARG, "problem %d: n (%d) must be a positive multiple of K (%d)", p, d.n, d.K);
    if (d.dim != 2 && d.dim != 3) return fail(OT_ERR_ARG, "problem %d: dim must be 2 or 3", p);
    if (!(d.eps > 0.0) || !std::isfinite(d.eps)) return fail(OT_ERR_ARG, "problem %d: eps must be > 0", p);
    if (!d.x || !d.y || !d.a || !d.b || !d.logK || !d.f || !d.g || !d.out)
      return fail(OT_ERR_ARG, "problem %d: x, y, a, b, logK, f, g and out must be non-NULL", p);
    if (d.n / d.K > 4096)
      return fail(OT_ERR_UNSUPPORTED, "problem %d: block size m = %d above 4096", p, d.n / d.K);
    const int lpr = d.tile_cfg & 0xff, fcb = (d.tile_cfg >> 8) & 0xff;
    if ((lpr != 0 && lpr != 16 && lpr != 32 && lpr != 64) || fcb > 16 || (d.tile_cfg >> 16) != 0)
      return fail(OT_ERR_ARG,
                  "problem %d: tile_cfg must be lanes (0, 16, 32, 64) | fold columns / 64 "
                  "(0 .. 16) << 8", p);
  }
  if (csot::batched_plan(h, count, plan) != 0) return fail(OT_ERR_UNSUPPORTED, "too many tiles");
  return ok();
}

size_t ot_batched_workspace_bytes(int32_t count) {
  return count > 0 ? csot::batched_ws_bytes(count) : 0;
}

int ot_sinkhorn_reduced_batched(const ot_batch_desc* descs, int32_t count, const int32_t* plan,
                                const int32_t* plan_host, const ot_opts* opts, void* ws,
                                size_t ws_bytes, void* stream) {
  if (!descs || !plan || !plan_host || count <= 0)
    return fail(OT_ERR_ARG, "descriptors, plan, plan_host and count > 0 required");
  ot_opts o = opts ? *opts : defaults();
  int rc = check_opts(o);
  if (rc) return rc;
  if ((rc = check_ws(ws, ws_bytes, csot::batched_ws_bytes(count)))) return rc;
  // every problem has at least one fold tile and one value tile
  if (plan_host[2] != count || plan_host[0] < count || plan_host[1] < count)
    return fail(OT_ERR_ARG, "plan_host is not ot_batched_plan's output for %d problems", count);
  hipError_t e = csot::launch_batched(descs, count, plan, plan_host, o.tol, o.max_iter,
                                      o.fold_fp64, o.warm_start, ws, static_cast<hipStream_t>(stream),
                                      static_cast<hipEvent_t*>(o.timing_events));
  if (e != hipSuccess) return hip_fail(e, "batched launch");
  return ok();
}

size_t ot_peaks_workspace_bytes(void) { return csot::peaks_scratch_bytes(); }

int ot_measure_peaks(double* out, void* ws, size_t ws_bytes, void* stream) {
  if (!out) return fail(OT_ERR_ARG, "out must be non-NULL");
  int rc = check_ws(ws, ws_bytes, csot::peaks_scratch_bytes());
  if (rc) return rc;
  hipError_t e = csot::measure_peaks(out, ws, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "peaks micro-benchmarks");
  return ok();
}

}  // extern "C"
