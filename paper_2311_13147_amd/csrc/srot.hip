// Cyclic strongly convex-regularised OT with the quadratic regulariser
// phi(x) = (lam / 2) x^2 (x >= 0): alternating maximisation of the reduced dual (Thm. 2,
// eq. dual_problem_cyclic_ROT), the algorithm of the C-SROT section.
//
// With z fixed, w_i is the root of eq. derivative_of_objective_function,
//   sum_{k,j} max(0, w_i + z_j - C_ijk) = lam alpha_i,
// a piecewise linear increasing function of w_i.  One workgroup per point runs Newton's method on
// it from the point's previous value: the slope is the number of active terms; from the left
// of the root the first step lands right of it (the function is convex), from there the
// iterates decrease monotonically and stop once the active set is right.  Costs are
// block-row 0's, from the coordinates (float32) or a dense C; every Newton step re-evaluates
// the K m terms of the point.  Columns (z with w fixed) likewise.
//
// The whole solve is one persistent launch (every workgroup resident at once): workgroup b
// owns points [b R, b R + R) of both sides and exchanges the potentials through epoch-tagged
// slots, as the reduced Sinkhorn solver does.  The first Newton evaluation of a row update
// starts at the row's previous w, so it yields that row's sum for the current state: its
// residual r_i = sum / lam - alpha_i is free.  Every workgroup publishes its sum of r_i^2 with
// its new w, stages all of them with the w exchange and takes the same stop decision on the
// state one half-iteration back (the full-space row residual sqrt(K) ||r||_2 <= tol); no host
// round trip inside the loop.  The float64 residuals are computed once, after the loop.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "launch.hpp"

namespace csot {

constexpr int kSrotWaves = 4;  // points per workgroup, one per wave

template <int DIM, bool ROW>
__device__ __forceinline__ float srot_cost(const Geom& g, int a, int b, int k) {
  // ROW: C_{a b k} (row a, column b); COL: C_{b a k} (row b, column a)
  const int i = ROW ? a : b, j = ROW ? b : a;
  if constexpr (DIM == 0) {
    return g.C[(int64_t)i * g.ldc + (int64_t)k * g.m + j];
  } else {
    const int64_t J = (int64_t)k * g.m + j;
    float c = 0.0f;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const float df = g.x[(int64_t)i * DIM + d] - g.y[J * DIM + d];
      c = fmaf(df, df, c);
    }
    return c;
  }
}

struct SrotParams {
  Geom g;
  float lam;
  double tol2;          // tol^2 / K (compared with sum r_i^2); 0: run max_iter iterations
  int max_iter, W, R;
  const float* alpha;   // [m] folded marginals
  const float* beta;
  float* w;             // [m] in: the start (zero or warm); out: the returned state
  float* z;
  uint64_t* wx;         // [mp] w slots: epoch t + 1 carries w^t
  uint64_t* zx;         // [mp] z slots: epoch t + 1 carries z^t (epoch 1: the start)
  uint64_t* rsx;        // [2][W] residual partials, double-buffered by iteration parity
  uint32_t* ctl;        // [0] abort flag, [1] flags raised (1 non-finite, 2 aborted wait)
  double* dstats;       // [0] iterations, [1] converged
};

constexpr int kSrotThreads = kWave * kSrotWaves;

// LDS partials of one Newton step, one entry per wave
struct SrotRed {
  double s64[kSrotWaves];
  float s[kSrotWaves], cnt[kSrotWaves], vmin[kSrotWaves];
};

// Sum, active count and minimum of the terms of one Newton step over the workgroup, through
// LDS; every thread returns the same totals (same order everywhere).  With FIRST the float64
// sum is reduced too.
template <bool FIRST>
__device__ __forceinline__ void srot_step_reduce(SrotRed* rd, float& s, float& cnt, float& vmin,
                                                 double& sd) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  s = wave_sum_all(s);
  cnt = wave_sum_all(cnt);
  vmin = -wave_max(-vmin);
  if (FIRST) sd = wave_sum_d(sd);
  if (lane == 0) {
    rd->s[wv] = s;
    rd->cnt[wv] = cnt;
    rd->vmin[wv] = vmin;
    if (FIRST) rd->s64[wv] = sd;
  }
  __syncthreads();
  s = 0.0f;
  cnt = 0.0f;
  vmin = INFINITY;
  sd = 0.0;
#pragma unroll
  for (int q = 0; q < kSrotWaves; ++q) {
    s += rd->s[q];
    cnt += rd->cnt[q];
    vmin = fminf(vmin, rd->vmin[q]);
    if (FIRST) sd += rd->s64[q];
  }
  __syncthreads();  // the partials are read before the next step overwrites them
}

// One Newton update of w from the step's totals; returns true once the root is reached (the
// active set is right, up to float32 rounding of the terms).  Left of every term (no active
// term) it moves to a point right of the root.
__device__ __forceinline__ bool srot_newton_update(float& w, float s, float cnt, float vmin,
                                                   float target) {
  if (cnt == 0.0f) {
    w = vmin + target;
    return false;
  }
  const float dw = (s - target) / cnt;
  w -= dw;
  return fabsf(dw) <= 2e-7f * (fabsf(w) + fabsf(vmin) + target);
}

// Newton's method on point a's equation against the other side's potential (staged in LDS),
// from `start`; returns the root.  With FIRST the first evaluation also sums the terms in
// float64, the way the residual kernel does, and *s64 receives that sum: lam times the point's
// plan marginal in the state the update starts from.  Every thread returns the same values.
//
// NV > 0: the K m terms v = C - other of the point are computed once into registers (NV per
// thread, K m <= NV kSrotThreads; +inf pads) and the Newton steps only scan them.  NV = 0:
// every step recomputes the terms (any K m).
template <int DIM, bool ROW, bool FIRST, int NV>
__device__ float srot_newton(const Geom& g, int a, float start, float target,
                             const float* __restrict__ other, SrotRed* rd, double* s64) {
  const int tid = threadIdx.x;
  float w = start;
  if constexpr (NV > 0) {
    float v[NV];
    double sd = 0.0;
    int k = 0, b = tid;
    while (b >= g.m) {
      b -= g.m;
      ++k;
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      v[i] = INFINITY;
      if (k < g.K) {
        const float c = srot_cost<DIM, ROW>(g, a, b, k), o = other[b];
        v[i] = c - o;
        if (FIRST) {
          const double y = (double)w + (double)o - (double)c;
          if (y > 0.0) sd += y;
        }
        b += kSrotThreads;
        while (b >= g.m) {
          b -= g.m;
          ++k;
        }
      }
    }
    for (int step = 0; step < 64; ++step) {
      float s = 0.0f, cnt = 0.0f, vmin = INFINITY;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const float d = w - v[i];
        if (d > 0.0f) {
          s += d;
          cnt += 1.0f;
        }
        vmin = fminf(vmin, v[i]);
      }
      if (FIRST && step == 0) {
        srot_step_reduce<true>(rd, s, cnt, vmin, sd);
        *s64 = sd;
      } else {
        double unused = 0.0;
        srot_step_reduce<false>(rd, s, cnt, vmin, unused);
      }
      if (srot_newton_update(w, s, cnt, vmin, target)) break;
    }
  } else {
    for (int step = 0; step < 64; ++step) {
      const bool first = FIRST && step == 0;
      float s = 0.0f, cnt = 0.0f, vmin = INFINITY;
      double sd = 0.0;
      for (int k = 0; k < g.K; ++k) {
        for (int b = tid; b < g.m; b += kSrotThreads) {
          const float c = srot_cost<DIM, ROW>(g, a, b, k), o = other[b];
          const float v = c - o;
          if (v < w) {
            s += w - v;
            cnt += 1.0f;
          }
          vmin = fminf(vmin, v);
          if (first) {
            const double y = (double)w + (double)o - (double)c;
            if (y > 0.0) sd += y;
          }
        }
      }
      if (first) {
        srot_step_reduce<true>(rd, s, cnt, vmin, sd);
        *s64 = sd;
      } else {
        srot_step_reduce<false>(rd, s, cnt, vmin, sd);
      }
      if (srot_newton_update(w, s, cnt, vmin, target)) break;
    }
  }
  return w;
}

// The persistent solver.  Iteration t: stage z^{t-1}; Newton for the own rows (its first
// evaluation gives their residuals in the state after t - 1 iterations); publish w^t and this
// workgroup's sum of squared residuals; stage w^t with every workgroup's sum; stop on the
// state after t - 1 iterations if it meets the tolerance (from t = 2 on, when z^{t-1} has
// been solved against w^{t-1}, so the column residuals are zero up to rounding) or if
// t - 1 = max_iter; otherwise Newton for the own columns and publish z^t.  Every workgroup
// sums the same partials in the same order, so all take the same decision.
template <int DIM, int NV>
__global__ void __launch_bounds__(kSrotThreads) srot_solver_kernel(SrotParams p) {
  extern __shared__ double lds_d[];
  const Geom& g = p.g;
  const int m = g.m, mp = (m + 3) & ~3;
  SrotRed* rd = reinterpret_cast<SrotRed*>(lds_d);
  float* Vs = reinterpret_cast<float*>(rd + 1);  // [mp] the other side's potential, staged
  float* wprev = Vs + mp;                        // [R] own rows' w before the last update
  float* wcur = wprev + p.R;                     // [R]
  float* zcur = wcur + p.R;                      // [R] own columns' z
  float* rsv = zcur + p.R;                       // [W] staged residual partials
  int* bad = reinterpret_cast<int*>(rsv + p.W);
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int r0 = blockIdx.x * p.R;
  const int nr = max(0, min(p.R, m - r0));
  uint32_t* abort_flag = p.ctl;
  for (int q = tid; q < nr; q += kSrotThreads) {
    const float w0 = p.w[r0 + q], z0 = p.z[r0 + q];
    wprev[q] = wcur[q] = w0;
    zcur[q] = z0;
    slot_publish(p.zx + r0 + q, z0, 1u);  // z^0
  }
  if (tid == 0) *bad = 0;
  __syncthreads();
  int iters = 0, converged = 0;
  uint32_t flags = 0;
  for (int t = 1;; ++t) {
    if (!stage_slots(p.zx, m, mp, (uint32_t)t, Vs, nullptr, 0, 0, nullptr, abort_flag, bad)) {
      flags |= 2u;
      break;
    }
    double racc = 0.0;
    for (int q = 0; q < nr; ++q) {
      const int a = r0 + q;
      double s64;
      const float wn = srot_newton<DIM, true, true, NV>(g, a, wcur[q], p.lam * p.alpha[a], Vs,
                                                        rd, &s64);
      const double r = s64 / (double)p.lam - (double)p.alpha[a];
      racc += r * r;
      if (tid == 0) {
        wprev[q] = wcur[q];
        wcur[q] = wn;
        slot_publish(p.wx + a, wn, (uint32_t)t + 1u);
      }
    }
    uint64_t* rs = p.rsx + (size_t)(t & 1) * p.W;
    if (tid == 0) slot_publish(rs + blockIdx.x, (float)racc, (uint32_t)t + 1u);
    if (!stage_slots(p.wx, m, mp, (uint32_t)t + 1u, Vs, rs, p.W, (uint32_t)t + 1u, rsv,
                     abort_flag, bad)) {
      flags |= 2u;
      break;
    }
    bool stop = t - 1 >= p.max_iter;
    if (t >= 2) {
      float sres = 0.0f;
      for (int v = lane; v < p.W; v += kWave) sres += rsv[v];
      sres = wave_sum_all(sres);
      const bool fin = sres == sres && sres <= 3.0e38f;
      converged = p.tol2 > 0.0 && fin && (double)sres <= p.tol2;
      if (!fin) flags |= 1u;
      stop = stop || converged || !fin;
    }
    if (stop) {
      iters = t - 1;
      break;
    }
    for (int q = 0; q < nr; ++q) {
      const int a = r0 + q;
      const float zn = srot_newton<DIM, false, false, NV>(g, a, zcur[q], p.lam * p.beta[a], Vs,
                                                          rd, nullptr);
      if (tid == 0) {
        zcur[q] = zn;
        slot_publish(p.zx + a, zn, (uint32_t)t + 1u);
      }
    }
  }
  // the state after `iters` iterations: w^{t-1} (wprev) and z^{t-1} (zcur)
  __syncthreads();
  for (int q = tid; q < nr; q += kSrotThreads) {
    p.w[r0 + q] = flags & 2u ? wcur[q] : wprev[q];
    p.z[r0 + q] = zcur[q];
  }
  if (blockIdx.x == 0 && tid == 0) {
    p.dstats[0] = (double)iters;
    p.dstats[1] = (double)converged;
  }
  if (tid == 0 && flags) atomicOr(p.ctl + 1, flags);
}

// Full-space L2 norms of the float64 residuals (out[0 .. m) rows, [m .. 2m) columns) into
// dstats[2], dstats[3]; dstats[5] = the flags the solver raised.
__global__ void __launch_bounds__(1024)
    srot_check_kernel(int m, int K, const double* __restrict__ res, const uint32_t* ctl,
                      double* __restrict__ dstats) {
  __shared__ double red[1024 / kWave];
  double er = 0.0, ec = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    er += res[i] * res[i];
    ec += res[m + i] * res[m + i];
  }
  er = block_sum_d(er, red);
  ec = block_sum_d(ec, red);
  if (threadIdx.x == 0) {
    dstats[2] = sqrt((double)K * er);
    dstats[3] = sqrt((double)K * ec);
    dstats[5] = (double)ctl[1];
  }
}

// Residual sums of the current plan T_ijk = max(0, w_i + z_j - C_ijk) / lam: out[a] =
// (sum over the other index and k) - marg[a], in float64.
template <int DIM, bool ROW>
__global__ void __launch_bounds__(kWave* kSrotWaves)
    srot_residual_kernel(Geom g, float lam, const float* __restrict__ wv,
                         const float* __restrict__ zv, const float* __restrict__ marg,
                         double* __restrict__ out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int a = blockIdx.x * kSrotWaves + threadIdx.x / kWave;
  if (a >= g.m) return;
  const double own = ROW ? wv[a] : zv[a];
  const float* other = ROW ? zv : wv;
  double s = 0.0;
  for (int k = 0; k < g.K; ++k)
    for (int b = lane; b < g.m; b += kWave) {
      const double y = own + (double)other[b] - (double)srot_cost<DIM, ROW>(g, a, b, k);
      if (y > 0.0) s += y;
    }
  s = wave_sum_d(s);
  if (lane == 0) out[a] = s / (double)lam - (double)marg[a];
}

__global__ void srot_init_kernel(Geom g, int warm, float* __restrict__ alpha,
                                 float* __restrict__ beta, float* __restrict__ w,
                                 float* __restrict__ z) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < g.m; i += gridDim.x * blockDim.x) {
    double sa = 0.0, sb = 0.0;
    for (int r = 0; r < g.K; ++r) {
      sa += (double)g.a[(int64_t)r * g.m + i];
      sb += (double)g.b[(int64_t)r * g.m + i];
    }
    alpha[i] = (float)(sa / g.K);
    beta[i] = (float)(sb / g.K);
    if (!warm) {
      w[i] = 0.0f;
      z[i] = 0.0f;
    }
  }
}

static size_t a256(size_t v) { return (v + 255) / 256 * 256; }

// Launch plan of the persistent solver: W workgroups of kSrotThreads, R points each, all
// resident at once.
struct SrotPlan {
  int W, R;
  size_t lds;
};

static size_t srot_lds_bytes(int m, int R, int W) {
  return sizeof(SrotRed) + sizeof(float) * ((size_t)((m + 3) & ~3) + 3 * (size_t)R + W) + 16;
}

// Registers per thread for the cached terms of a point (0: recompute every Newton step).
static int srot_nv(const Geom& g) {
  const long km = (long)g.K * g.m;
  return km <= 8L * kSrotThreads ? 8 : km <= 32L * kSrotThreads ? 32
                                     : km <= 64L * kSrotThreads ? 64 : 0;
}

template <int DIM>
static const void* srot_kernel_nv(int nv) {
  switch (nv) {
    case 8: return (const void*)srot_solver_kernel<DIM, 8>;
    case 32: return (const void*)srot_solver_kernel<DIM, 32>;
    case 64: return (const void*)srot_solver_kernel<DIM, 64>;
    default: return (const void*)srot_solver_kernel<DIM, 0>;
  }
}

static const void* srot_kernel(const Geom& g) {
  const int nv = srot_nv(g);
  return g.dim == 0 ? srot_kernel_nv<0>(nv) : g.dim == 2 ? srot_kernel_nv<2>(nv)
                                                         : srot_kernel_nv<3>(nv);
}

static bool plan_srot(const Geom& g, SrotPlan* pl) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return false;
  const void* k = srot_kernel(g);
  // one point per workgroup while they fit co-resident, otherwise R points each (a larger R
  // needs a little more LDS, hence the loop)
  constexpr size_t kLdsLimit = 64 * 1024;  // the default dynamic LDS limit of a launch
  int R = 1;
  for (int pass = 0; pass < 16; ++pass) {
    const int W = (g.m + R - 1) / R;
    const size_t lds = srot_lds_bytes(g.m, R, W);
    int next = R + 1;
    if (lds <= kLdsLimit) {
      int per_cu = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kSrotThreads, lds) !=
          hipSuccess)
        return false;
      const long cap = (long)per_cu * cus;
      if (cap > 0 && W <= cap) {
        pl->W = W;
        pl->R = R;
        pl->lds = lds;
        return true;
      }
      if (cap > 0) next = std::max(next, (int)((g.m + cap - 1) / cap));
    } else if (srot_lds_bytes(g.m, 1, 1) > kLdsLimit) {
      return false;  // the staged potential alone exceeds the limit
    }
    R = next;
  }
  return false;
}

// workspace: alpha[m] | beta[m] | res[2m] doubles | dstats[8] doubles | ctl[64 words] |
// wx[mp] | zx[mp] | rsx[2W] (64-bit slots; W <= m)
size_t srot_ws_bytes(const Geom& g) {
  const int mp = (g.m + 3) & ~3;
  return 2 * a256(sizeof(float) * g.m) + a256(sizeof(double) * 2 * g.m) + a256(64) + a256(256) +
         2 * a256(sizeof(uint64_t) * mp) + a256(sizeof(uint64_t) * 2 * g.m);
}

template <int DIM>
static hipError_t srot_residuals(const Geom& g, float lam, const float* alpha,
                                 const float* beta, const float* w, const float* z,
                                 double* out, hipStream_t s) {
  const dim3 grid((g.m + kSrotWaves - 1) / kSrotWaves), block(kWave * kSrotWaves);
  hipLaunchKernelGGL((srot_residual_kernel<DIM, true>), grid, block, 0, s, g, lam, w, z, alpha,
                     out);
  hipLaunchKernelGGL((srot_residual_kernel<DIM, false>), grid, block, 0, s, g, lam, w, z, beta,
                     out + g.m);
  return hipGetLastError();
}

bool srot_supported(const Geom& g) {
  SrotPlan pl;
  return plan_srot(g, &pl);
}

// One persistent launch for the iterations (the stop test on the device), then the float64
// residuals and their norms; res [host] receives {iterations, converged, err_row, err_col, -,
// flags} through one copy and one stream synchronisation at the end.
hipError_t run_srot(const Geom& g, double lam, double tol, int max_iter, int warm, float* w,
                    float* z, void* ws, double* res, hipStream_t s) {
  SrotPlan pl;
  if (!plan_srot(g, &pl)) return hipErrorInvalidConfiguration;
  const int mp = (g.m + 3) & ~3;
  char* base = static_cast<char*>(ws);
  size_t off = 0;
  float* alpha = reinterpret_cast<float*>(base + off); off += a256(sizeof(float) * g.m);
  float* beta = reinterpret_cast<float*>(base + off); off += a256(sizeof(float) * g.m);
  double* rsd = reinterpret_cast<double*>(base + off); off += a256(sizeof(double) * 2 * g.m);
  double* dstats = reinterpret_cast<double*>(base + off); off += a256(64);
  uint32_t* ctl = reinterpret_cast<uint32_t*>(base + off); off += a256(256);
  uint64_t* wx = reinterpret_cast<uint64_t*>(base + off); off += a256(sizeof(uint64_t) * mp);
  uint64_t* zx = reinterpret_cast<uint64_t*>(base + off); off += a256(sizeof(uint64_t) * mp);
  uint64_t* rsx = reinterpret_cast<uint64_t*>(base + off); off += a256(sizeof(uint64_t) * 2 * g.m);
  const int ib = (g.m + 255) / 256 < 1024 ? (g.m + 255) / 256 : 1024;
  hipLaunchKernelGGL(srot_init_kernel, dim3(ib), dim3(256), 0, s, g, warm, alpha, beta, w, z);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // statistics, control words and slots: epochs start at 1, so zeroed slots are never current
  const size_t zero_bytes = off - ((char*)dstats - base);
  if ((e = launch_zero_words(reinterpret_cast<uint32_t*>(dstats), (int)(zero_bytes / 4), s)) !=
      hipSuccess)
    return e;
  SrotParams p;
  p.g = g;
  p.lam = (float)lam;
  p.tol2 = tol * tol / (double)g.K;
  p.max_iter = max_iter;
  p.W = pl.W;
  p.R = pl.R;
  p.alpha = alpha;
  p.beta = beta;
  p.w = w;
  p.z = z;
  p.wx = wx;
  p.zx = zx;
  p.rsx = rsx;
  p.ctl = ctl;
  p.dstats = dstats;
  // an ordinary launch: the plan admits no more workgroups than are resident at once, and
  // every wait is bounded (a timed-out wait raises the abort flag, which ends every loop)
  void* args[] = {&p};
  if ((e = hipLaunchKernel(srot_kernel(g), dim3(pl.W), dim3(kSrotThreads), args, pl.lds, s)) !=
      hipSuccess)
    return e;
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const float fl = (float)lam;
  switch (g.dim) {
    case 0: e = srot_residuals<0>(g, fl, alpha, beta, w, z, rsd, s); break;
    case 2: e = srot_residuals<2>(g, fl, alpha, beta, w, z, rsd, s); break;
    default: e = srot_residuals<3>(g, fl, alpha, beta, w, z, rsd, s); break;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(srot_check_kernel, dim3(1), dim3(1024), 0, s, g.m, g.K, rsd, ctl, dstats);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(res, dstats, 6 * sizeof(double), hipMemcpyDeviceToHost, s)) !=
      hipSuccess)
    return e;
  return hipStreamSynchronize(s);
}

}  // namespace csot
