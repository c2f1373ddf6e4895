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
#include <cmath>
#include <vector>

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

// One workgroup of kSrotWaves waves per point: its threads split the K m terms, and the
// partial sums of a Newton step are combined through LDS, so that a step costs K m / 256 terms
// per thread (the cyclic problem has only m points to spread over the chip).
template <int DIM, bool ROW>
__global__ void __launch_bounds__(kWave* kSrotWaves)
    srot_update_kernel(Geom g, float lam, const float* __restrict__ other,
                       const float* __restrict__ marg, float* __restrict__ own) {
  __shared__ float ps[kSrotWaves], pc[kSrotWaves], pm[kSrotWaves];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const int a = blockIdx.x;
  const float target = lam * marg[a];
  float w = own[a];
  for (int step = 0; step < 64; ++step) {
    float s = 0.0f, cnt = 0.0f, vmin = INFINITY;
    for (int k = 0; k < g.K; ++k) {
      for (int b = tid; b < g.m; b += kWave * kSrotWaves) {
        const float v = srot_cost<DIM, ROW>(g, a, b, k) - other[b];
        if (v < w) {
          s += w - v;
          cnt += 1.0f;
        }
        vmin = fminf(vmin, v);
      }
    }
    s = wave_sum_all(s);
    cnt = wave_sum_all(cnt);
    vmin = -wave_max(-vmin);
    if (lane == 0) {
      ps[wv] = s;
      pc[wv] = cnt;
      pm[wv] = vmin;
    }
    __syncthreads();
    s = 0.0f;
    cnt = 0.0f;
    vmin = INFINITY;
#pragma unroll
    for (int q = 0; q < kSrotWaves; ++q) {  // the same order in every thread
      s += ps[q];
      cnt += pc[q];
      vmin = fminf(vmin, pm[q]);
    }
    __syncthreads();  // the partials are read before the next step overwrites them
    if (cnt == 0.0f) {  // left of every term: move to a point right of the root
      w = vmin + target;
      continue;
    }
    const float dw = (s - target) / cnt;
    w -= dw;
    // the root is reached (the active set is right) up to float32 rounding of the terms
    if (fabsf(dw) <= 2e-7f * (fabsf(w) + fabsf(vmin) + target)) break;
  }
  if (tid == 0) own[a] = w;
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

size_t srot_ws_bytes(const Geom& g) {
  return 2 * a256(sizeof(float) * g.m) + a256(sizeof(double) * 2 * g.m);
}

template <int DIM>
static hipError_t srot_step(const Geom& g, float lam, const float* alpha, const float* beta,
                            float* w, float* z, hipStream_t s) {
  const dim3 grid(g.m), block(kWave * kSrotWaves);  // one workgroup per point
  hipLaunchKernelGGL((srot_update_kernel<DIM, true>), grid, block, 0, s, g, lam, z, alpha, w);
  hipLaunchKernelGGL((srot_update_kernel<DIM, false>), grid, block, 0, s, g, lam, w, beta, z);
  return hipGetLastError();
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

// Host loop: an iteration is the w-update then the z-update (two launches); every
// check_every iterations (tol > 0; else after the last) the float64 residuals are copied back
// and the loop stops when the full-space row residual sqrt(K) ||T 1 - alpha|| is at most tol
// (the column residual is zero up to rounding after the z-update).  Synchronises at every
// check.
hipError_t run_srot(const Geom& g, double lam, double tol, int max_iter, int check_every,
                    int warm, float* w, float* z, void* ws, hipStream_t s, double* res) {
  char* base = static_cast<char*>(ws);
  float* alpha = reinterpret_cast<float*>(base);
  float* beta = reinterpret_cast<float*>(base + a256(sizeof(float) * g.m));
  double* rsd = reinterpret_cast<double*>(base + 2 * a256(sizeof(float) * g.m));
  const int ib = (g.m + 255) / 256 < 1024 ? (g.m + 255) / 256 : 1024;
  hipLaunchKernelGGL(srot_init_kernel, dim3(ib), dim3(256), 0, s, g, warm, alpha, beta, w, z);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  std::vector<double> h(2 * (size_t)g.m);
  const float fl = (float)lam;
  int it = 0;
  double er = INFINITY, ec = INFINITY;
  bool conv = false;
  const int every = check_every > 0 ? check_every : 1;
  while (it < max_iter) {
    switch (g.dim) {
      case 0: e = srot_step<0>(g, fl, alpha, beta, w, z, s); break;
      case 2: e = srot_step<2>(g, fl, alpha, beta, w, z, s); break;
      case 3: e = srot_step<3>(g, fl, alpha, beta, w, z, s); break;
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    ++it;
    // tol = 0 asks for max_iter iterations: the residuals are needed only for the statistics
    if ((tol > 0.0 && it % every == 0) || it == max_iter) {
      switch (g.dim) {
        case 0: e = srot_residuals<0>(g, fl, alpha, beta, w, z, rsd, s); break;
        case 2: e = srot_residuals<2>(g, fl, alpha, beta, w, z, rsd, s); break;
        default: e = srot_residuals<3>(g, fl, alpha, beta, w, z, rsd, s); break;
      }
      if (e != hipSuccess) return e;
      if ((e = hipMemcpyAsync(h.data(), rsd, sizeof(double) * 2 * g.m, hipMemcpyDeviceToHost,
                              s)) != hipSuccess)
        return e;
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
      double sr = 0.0, sc = 0.0;
      for (int i = 0; i < g.m; ++i) {
        sr += h[i] * h[i];
        sc += h[g.m + i] * h[g.m + i];
      }
      er = std::sqrt((double)g.K * sr);
      ec = std::sqrt((double)g.K * sc);
      if (tol > 0.0 && er <= tol) {
        conv = true;
        break;
      }
    }
  }
  res[0] = it;
  res[1] = conv ? 1.0 : 0.0;
  res[2] = er;
  res[3] = ec;
  return hipSuccess;
}

}  // namespace csot
