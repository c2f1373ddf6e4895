// Many independent reduced problems of uneven size in one stream of four launches, all
// capturable in a HIP graph (no host synchronisation, no memset, no allocation):
//
//   1. fold   : tiles of 16 rows of one problem -> logK (base 2) and its transpose, alpha, beta
//               (eq. def_Kij; Alg. 3 stage-1 averaging of the marginals);
//   2. solve  : ONE persistent launch; each workgroup pops the next problem from a device work
//               queue (largest first) and runs the cyclic Sinkhorn loop of Alg. 2 on it alone,
//               synchronising only within the workgroup; logK stays in LDS when it fits;
//   3. values : tiles of 16 rows (or columns) of one problem -> objective terms, gradients of
//               the first block's points, float64 marginal sums;
//   4. finalize per problem: P, D, <C,T>, errors.
//
// Per problem the cost is block-row 0's: C_ijk = |x_i - y_{k m + j}|^2.  Gradients are with
// respect to the first block's points (x_i, y_j for i, j < m) of the full problem:
//   dx_i = 2 sum_{k,j} T_ijk (x_i - y_{k m + j}),
//   dy_j = 2 sum_{r,i} T_{i j ((K - r) mod K)} (y_j - x_{r m + i}),
// exactly the first m rows of the single-problem gradients (the other blocks' rows follow
// from the cyclic symmetry of the data).
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "launch.hpp"
#include "csot.h"

namespace csot {

constexpr int kBT = 16;            // rows (or columns) per fold / values tile
constexpr int kBSolveThreads = 1024;
constexpr int kBSolveWaves = kBSolveThreads / kWave;
constexpr int kBMaxLds = 148 * 1024;

__device__ __forceinline__ int find_problem(const int32_t* __restrict__ start, int count, int b) {
  int lo = 0, hi = count - 1;  // largest p with start[p] <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ float* bscratch_L(const ot_batch_desc& d) { return d.logK; }
__device__ __forceinline__ int bm(const ot_batch_desc& d) { return d.n / d.K; }

template <int DIM, typename Real>
__device__ __forceinline__ Real bcost(const float* __restrict__ x, int I,
                                      const float* __restrict__ y, int J) {
  Real c = 0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const Real df = (Real)x[(int64_t)I * DIM + d] - (Real)y[(int64_t)J * DIM + d];
    c += df * df;
  }
  return c;
}

// ---- 1. fold -------------------------------------------------------------------------------
template <int DIM>
__device__ void fold_tile(const ot_batch_desc& d, int i0, int fp64_mode) {
  const int m = bm(d), K = d.K;
  float* L = d.logK;
  float* LT = L + (size_t)m * m;
  const bool fp64 = fp64_mode == 1 || (fp64_mode == -1 && K >= 32);
  const double ie = 1.0 / d.eps;
  const int rows = min(kBT, m - i0);
  for (int e = threadIdx.x; e < rows * m; e += blockDim.x) {
    const int i = i0 + e / m, j = e - (e / m) * m;
    float v;
    if (fp64) {
      double cmin = 1.0e300;
      for (int k = 0; k < K; ++k) cmin = fmin(cmin, bcost<DIM, double>(d.x, i, d.y, k * m + j));
      double s = 0.0;
      for (int k = 0; k < K; ++k) s += exp((cmin - bcost<DIM, double>(d.x, i, d.y, k * m + j)) * ie);
      v = (float)((-cmin * ie + log(s)) * kLog2eD);
    } else {
      const float s2 = (float)(kLog2eD * ie);
      float cmin = 3.0e38f;
      for (int k = 0; k < K; ++k) cmin = fminf(cmin, bcost<DIM, float>(d.x, i, d.y, k * m + j));
      float s = 0.0f;
      for (int k = 0; k < K; ++k) s += exp2_fast((cmin - bcost<DIM, float>(d.x, i, d.y, k * m + j)) * s2);
      v = -cmin * s2 + log2_fast(s);
    }
    L[(size_t)i * m + j] = v;
    LT[(size_t)j * m + i] = v;
  }
  if (i0 == 0) {  // folded marginals
    float* al = LT + (size_t)m * m;
    float* be = al + m;
    for (int i = threadIdx.x; i < 2 * m; i += blockDim.x) {
      const float* v = i < m ? d.a : d.b;
      const int ii = i < m ? i : i - m;
      double acc = 0.0;
      for (int r = 0; r < K; ++r) acc += (double)v[(int64_t)r * m + ii];
      (i < m ? al : be)[ii] = (float)(acc / K);
    }
  }
}

__global__ void __launch_bounds__(256)
    batched_fold_kernel(const ot_batch_desc* __restrict__ descs, int count,
                        const int32_t* __restrict__ tile_start, int fp64_mode) {
  const int p = find_problem(tile_start, count, blockIdx.x);
  const ot_batch_desc d = descs[p];
  const int i0 = (blockIdx.x - tile_start[p]) * kBT;
  if (i0 >= bm(d)) return;
  if (d.dim == 3) fold_tile<3>(d, i0, fp64_mode);
  else fold_tile<2>(d, i0, fp64_mode);
}

// ---- 2. solve ------------------------------------------------------------------------------
// LSE2 of (row[j] + vec[j]) over j < m by a group of LPR lanes (every lane gets the result).
template <int LPR>
__device__ __forceinline__ float grp_reduce_max(float v) {
  v = fmaxf(v, dpp_f32<kDppXor1>(v));
  v = fmaxf(v, dpp_f32<kDppXor2>(v));
  v = fmaxf(v, dpp_f32<kDppHalfMirror>(v));
  v = fmaxf(v, dpp_f32<kDppMirror>(v));
  if constexpr (LPR >= 32) v = fmaxf(v, __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F)));
  if constexpr (LPR == 64) v = fmaxf(v, __shfl_xor(v, 32, kWave));
  return v;
}
template <int LPR>
__device__ __forceinline__ float grp_reduce_sum(float v) {
  v += dpp_f32<kDppXor1>(v);
  v += dpp_f32<kDppXor2>(v);
  v += dpp_f32<kDppHalfMirror>(v);
  v += dpp_f32<kDppMirror>(v);
  if constexpr (LPR >= 32) v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
  if constexpr (LPR == 64) v += __shfl_xor(v, 32, kWave);
  return v;
}

template <int LPR>
__device__ __forceinline__ float grp_lse2(const float* row, const float* vec, int m, int gl) {
  float M = kNegBig;
  for (int j = gl; j < m; j += LPR) M = fmaxf(M, row[j] + vec[j]);
  M = grp_reduce_max<LPR>(M);
  float S = 0.0f;
  for (int j = gl; j < m; j += LPR) S += exp2_fast(row[j] + vec[j] - M);
  S = grp_reduce_sum<LPR>(S);
  return M + log2_fast(S);
}

struct BSolveArgs {
  const ot_batch_desc* descs;
  int count;
  const int32_t* order;   // problems, largest first
  uint32_t* queue;        // [0] next position, zeroed before the launch
  double tol;
  int max_iter;
  int warm;
};

template <int LPR>
__device__ void solve_one(const ot_batch_desc& d, const BSolveArgs& a, float* lds,
                          size_t lds_floats, float* red) {
  const int m = bm(d), K = d.K;
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int gl = lane % LPR, grp = tid / LPR, ngrp = kBSolveThreads / LPR;
  // LDS: F, Fprev, G, la2, lb2, al (m each) [+ L, LT when they fit]
  float* F = lds;
  float* Fp = F + m;
  float* G = Fp + m;
  float* la2 = G + m;
  float* lb2 = la2 + m;
  float* al = lb2 + m;
  float* gL = d.logK;
  float* gLT = gL + (size_t)m * m;
  const float* galpha = gLT + (size_t)m * m;
  const float* gbeta = galpha + m;
  const bool in_lds = (size_t)6 * m + (size_t)2 * m * m <= lds_floats;
  const float* L = gL;
  const float* LT = gLT;
  if (in_lds) {
    float* Ls = al + m;
    float* LTs = Ls + (size_t)m * m;
    for (int e = tid; e < m * m; e += blockDim.x) { Ls[e] = gL[e]; LTs[e] = gLT[e]; }
    L = Ls;
    LT = LTs;
  }
  const float s2 = (float)(kLog2eD / d.eps);
  for (int i = tid; i < m; i += blockDim.x) {
    la2[i] = log2f(galpha[i]);
    lb2[i] = log2f(gbeta[i]);
    al[i] = galpha[i];
    G[i] = a.warm ? d.g[i] * s2 : 0.0f;
    F[i] = 0.0f;
    Fp[i] = 0.0f;
  }
  __syncthreads();
  const double tol2 = a.tol * a.tol / (double)K;
  int iters = 0, converged = 0, flags = 0;
  for (int t = 1;; ++t) {
    // row update F^t from G^{t-1}; residual of the state after t-1
    float racc = 0.0f;
    for (int i = grp; i < m; i += ngrp) {
      const float Fn = la2[i] - grp_lse2<LPR>(L + (size_t)i * m, G, m, gl);
      if (gl == 0) {
        if (t >= 2) {
          const float rr = scaled_exp2m1(al[i], F[i] - Fn);
          racc += rr * rr;
        }
        Fp[i] = F[i];
        F[i] = Fn;
      }
    }
    racc = wave_sum_all(racc);
    if (lane == 0) red[tid / kWave] = racc;
    __syncthreads();
    if (t >= 2) {
      float s = 0.0f;
      for (int w = 0; w < kBSolveWaves; ++w) s += red[w];  // same order in every thread
      const bool fin = s == s && s < 3.0e38f;
      const bool conv = fin && (double)s <= tol2;
      if ((conv && tol2 > 0.0) || !fin || t - 1 >= a.max_iter) {
        iters = t - 1;
        converged = conv;
        flags = fin ? 0 : 1;
        break;  // uniform: every thread evaluated the same s
      }
    }
    __syncthreads();
    // column update G^t from F^t
    for (int j = grp; j < m; j += ngrp) {
      const float Gn = lb2[j] - grp_lse2<LPR>(LT + (size_t)j * m, F, m, gl);
      if (gl == 0) G[j] = Gn;
    }
    __syncthreads();
  }
  // outputs: the state after iteration `iters` = (Fp, G)
  const float to_nat = (float)(d.eps * kLn2D);
  for (int i = tid; i < m; i += blockDim.x) {
    d.f[i] = Fp[i] * to_nat;
    d.g[i] = G[i] * to_nat;
  }
  if (tid == 0) {
    d.out[5] = (double)iters;
    d.out[6] = (double)converged;
    d.out[7] = (double)flags;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kBSolveThreads) batched_solve_kernel(BSolveArgs a) {
  extern __shared__ float4 lds4[];
  float* lds = reinterpret_cast<float*>(lds4);
  __shared__ float red[kBSolveWaves];
  __shared__ int s_p;
  const size_t lds_floats = (size_t)kBMaxLds / sizeof(float);
  for (;;) {
    if (threadIdx.x == 0) {
      const uint32_t pos = __hip_atomic_fetch_add(a.queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_p = pos < (uint32_t)a.count ? a.order[pos] : -1;
    }
    __syncthreads();
    const int p = s_p;
    __syncthreads();
    if (p < 0) return;  // queue drained: every workgroup reaches this
    const ot_batch_desc d = a.descs[p];
    const int m = bm(d);
    const int lpr = d.tile_cfg == 16 || d.tile_cfg == 32 || d.tile_cfg == 64
                        ? d.tile_cfg : (m >= 512 ? 64 : m >= 128 ? 32 : 16);
    if (lpr == 64) solve_one<64>(d, a, lds, lds_floats, red);
    else if (lpr == 32) solve_one<32>(d, a, lds, lds_floats, red);
    else solve_one<16>(d, a, lds, lds_floats, red);
  }
}

// ---- 3. values, gradients and float64 marginal sums ----------------------------------------
// Tiles [0, nrow) of a problem are row tiles, [nrow, 2 nrow) column tiles (16 points each).
// acc[p]: {P, <C,T>, mass, sum (rowsum - alpha)^2, sum (colsum - beta)^2, <f,alpha>, <g,beta>}
template <int DIM, bool ROW>
__device__ void values_tile(const ot_batch_desc& d, int a0, double* __restrict__ acc) {
  const int m = bm(d), K = d.K;
  const float* L = d.logK;
  const float* LT = L + (size_t)m * m;
  const float* al = LT + (size_t)m * m;
  const float* be = al + m;
  const float s2 = (float)(kLog2eD / d.eps);
  const float eps = (float)d.eps;
  const double ie = 1.0 / d.eps;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;  // 4 waves x 4 points
  double vP = 0.0, vC = 0.0, vM = 0.0, v2 = 0.0, vd = 0.0;
  for (int q = 0; q < 4; ++q) {
    const int A = a0 + wv * 4 + q;  // own point (row i or column j) in [0, m)
    if (A >= m) break;
    float po[DIM];
#pragma unroll
    for (int dd = 0; dd < DIM; ++dd) po[dd] = (ROW ? d.x : d.y)[(int64_t)A * DIM + dd];
    const float pa = ROW ? d.f[A] : d.g[A];
    float gacc[DIM];
#pragma unroll
    for (int dd = 0; dd < DIM; ++dd) gacc[dd] = 0.0f;
    float tP = 0.0f, tC = 0.0f, tM = 0.0f;
    for (int k = 0; k < K; ++k) {
      // ROW: partner column k m + b (block-row 0); COL: partner row r m + b with r = (K-k)%K
      const int r = (K - k) % K;
      for (int b = lane; b < m; b += kWave) {
        const int i = ROW ? A : b, j = ROW ? b : A;
        const float c = bcost<DIM, float>(d.x, i, d.y, k * m + j);
        const float fg = pa + (ROW ? d.g[b] : d.f[b]);
        const float T = exp2_fast((fg - c) * s2);
        const int P = ROW ? k * m + b : r * m + b;  // partner point for the gradient weight
#pragma unroll
        for (int dd = 0; dd < DIM; ++dd)
          gacc[dd] = fmaf(T, po[dd] - (ROW ? d.y : d.x)[(int64_t)P * DIM + dd], gacc[dd]);
        if (ROW) {
          const float z = (fg - c) / eps;
          tP = fmaf(T, c + eps * (z - 1.0f), tP);
          tC = fmaf(T, c, tC);
          tM += T;
        }
      }
    }
    // float64 marginal sum of own point A from logK
    double ms = 0.0;
    const float* Lrow = (ROW ? L : LT) + (size_t)A * m;
    for (int b = lane; b < m; b += kWave)
      ms += exp((double)Lrow[b] * kLn2D + ((double)pa + (double)(ROW ? d.g[b] : d.f[b])) * ie);
    ms = wave_sum_d(ms);
    const double target = ROW ? (double)al[A] : (double)be[A];
#pragma unroll
    for (int dd = 0; dd < DIM; ++dd) {
      const float gsum = wave_sum(gacc[dd]);
      float* dst = ROW ? d.dx : d.dy;
      if (lane == 0 && dst) dst[(int64_t)A * DIM + dd] = 2.0f * gsum;
    }
    if (ROW) {
      vP += wave_sum_d((double)tP);
      vC += wave_sum_d((double)tC);
      vM += wave_sum_d((double)tM);
    }
    v2 += (ms - target) * (ms - target);
    vd += (double)pa * target;
  }
  if (lane == 0) {
    if (ROW) {
      atomicAdd(&acc[0], vP);
      atomicAdd(&acc[1], vC);
      atomicAdd(&acc[2], vM);
      atomicAdd(&acc[3], v2);
      atomicAdd(&acc[5], vd);
    } else {
      atomicAdd(&acc[4], v2);
      atomicAdd(&acc[6], vd);
    }
  }
}

__global__ void __launch_bounds__(256)
    batched_values_kernel(const ot_batch_desc* __restrict__ descs, int count,
                          const int32_t* __restrict__ tile_start, double* __restrict__ accs) {
  const int p = find_problem(tile_start, count, blockIdx.x);
  const ot_batch_desc d = descs[p];
  const int m = bm(d);
  const int nrow = (m + kBT - 1) / kBT;
  const int t = blockIdx.x - tile_start[p];
  double* acc = accs + 8 * (size_t)p;
  const bool row = t < nrow;
  const int a0 = (row ? t : t - nrow) * kBT;
  if (d.dim == 3) { if (row) values_tile<3, true>(d, a0, acc); else values_tile<3, false>(d, a0, acc); }
  else { if (row) values_tile<2, true>(d, a0, acc); else values_tile<2, false>(d, a0, acc); }
}

__global__ void batched_finalize_kernel(const ot_batch_desc* __restrict__ descs, int count,
                                        const double* __restrict__ accs) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  const ot_batch_desc d = descs[p];
  const double* acc = accs + 8 * (size_t)p;
  const double K = d.K;
  d.out[0] = K * acc[0];
  d.out[1] = K * (acc[5] + acc[6]) - d.eps * K * acc[2];
  d.out[2] = K * acc[1];
  d.out[3] = sqrt(K * acc[3]);
  d.out[4] = sqrt(K * acc[4]);
}

__global__ void zero_d_words(double* p, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// ---- host ----------------------------------------------------------------------------------
static size_t a256(size_t v) { return (v + 255) / 256 * 256; }

size_t batched_plan_len(int count) { return 4 + 3 * (size_t)count; }

// plan = {nfold, nval, count, 0, order[count], fold_start[count], val_start[count]}
int batched_plan(const ot_batch_desc* h, int count, int32_t* plan) {
  std::vector<int> idx(count);
  for (int p = 0; p < count; ++p) idx[p] = p;
  auto cost = [&](int p) {
    const double m = (double)h[p].n / h[p].K;
    return m * m * (1.0 + 0.05 * h[p].K);  // iterations ~ m^2 each; fold ~ K m^2 once
  };
  std::stable_sort(idx.begin(), idx.end(), [&](int u, int v) { return cost(u) > cost(v); });
  int32_t* order = plan + 4;
  int32_t* fstart = order + count;
  int32_t* vstart = fstart + count;
  int64_t nf = 0, nv = 0;
  for (int p = 0; p < count; ++p) {
    order[p] = idx[p];
    const int m = h[p].n / h[p].K;
    const int tiles = (m + kBT - 1) / kBT;
    fstart[p] = (int32_t)nf;
    vstart[p] = (int32_t)nv;
    nf += tiles;
    nv += 2 * tiles;
  }
  if (nf > INT32_MAX || nv > INT32_MAX) return -1;
  plan[0] = (int32_t)nf;
  plan[1] = (int32_t)nv;
  plan[2] = count;
  plan[3] = 0;
  return 0;
}

size_t batched_ws_bytes(int count) { return a256(256) + a256(sizeof(double) * 8 * (size_t)count); }

hipError_t launch_batched(const ot_batch_desc* descs, int count, const int32_t* dplan,
                          int nfold, int nval, double tol, int max_iter, int fold_fp64,
                          int warm, void* ws, hipStream_t s) {
  char* base = static_cast<char*>(ws);
  uint32_t* queue = reinterpret_cast<uint32_t*>(base);
  double* accs = reinterpret_cast<double*>(base + a256(256));
  hipError_t e = launch_zero_words(queue, 64, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(zero_d_words, dim3(64), dim3(256), 0, s, accs, (int64_t)8 * count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int32_t* order = dplan + 4;
  const int32_t* fstart = order + count;
  const int32_t* vstart = fstart + count;
  hipLaunchKernelGGL(batched_fold_kernel, dim3(nfold), dim3(256), 0, s, descs, count, fstart,
                     fold_fp64);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  static bool attr = false;
  if (!attr) {
    if ((e = hipFuncSetAttribute((const void*)batched_solve_kernel,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kBMaxLds)) != hipSuccess)
      return e;
    attr = true;
  }
  int dev = 0, cus = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  BSolveArgs a{descs, count, order, queue, tol, max_iter, warm};
  const int grid = count < cus ? count : cus;
  hipLaunchKernelGGL(batched_solve_kernel, dim3(grid), dim3(kBSolveThreads), kBMaxLds, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(batched_values_kernel, dim3(nval), dim3(256), 0, s, descs, count, vstart, accs);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(batched_finalize_kernel, dim3((count + 255) / 256), dim3(256), 0, s, descs,
                     count, accs);
  return hipGetLastError();
}

}  // namespace csot
