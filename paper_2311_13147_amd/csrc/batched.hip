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
constexpr int kMaxGangF = 32;      // largest gang (workgroups cooperating on one problem)

__device__ __forceinline__ int find_problem(const int32_t* __restrict__ start, int count, int b) {
  int lo = 0, hi = count - 1;  // largest p with start[p] <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int bm(const ot_batch_desc& d) { return d.n / d.K; }
// scratch rows are padded to a multiple of 4 floats (16-byte aligned float4 loads)
__device__ __forceinline__ int bmp(int m) { return (m + 3) & ~3; }

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
// A tile is 16 rows of one problem; a thread owns one column j and 4 of the rows, so each
// y_{k m + j} it loads feeds 4 cost evaluations.  Two passes over k: the minimum cost per row,
// then the shifted exponential sum.  fp64 (default): costs, minimum and shifted exponents in
// float64, exponentials of the (non-positive) shifted exponents in float32 -- logK accurate
// to float32 rounding; otherwise all float32.  Output in base 2 (log2 of the folded kernel).
constexpr int kFoldQ = 4;  // rows per thread

constexpr int kFoldJC = 64;  // target columns j per LDS staging (one per lane of a wave)
constexpr int kFoldKC = 32;  // shifts k per LDS staging

// A fold tile: rows [i0, i0 + rows) (four groups of kFoldQ rows, one group per wave) against
// every column j.  For each chunk of 64 columns the target points y_{k m + j} of up to 32
// shifts are staged in LDS (K <= 32: one staging serves both passes), so each cost is an LDS
// read and a few FMAs and every staged point serves the tile's 16 rows.
template <int DIM, typename Real>
__device__ __forceinline__ void fold_cols(const ot_batch_desc& d, int i0, int rows, float* L,
                                          float* LT, float* __restrict__ ys) {
  const int m = bm(d), K = d.K, mp = bmp(m);
  const Real s2 = (Real)(kLog2eD / d.eps);
  const int tj = threadIdx.x % kFoldJC, grp = threadIdx.x / kFoldJC;
  const int ib = i0 + grp * kFoldQ;
  const bool grp_active = ib < i0 + rows;  // inactive groups still stage and meet barriers
  float xf[kFoldQ][DIM];
  Real xq[kFoldQ][DIM];
#pragma unroll
  for (int q = 0; q < kFoldQ; ++q) {
    const int i = min(ib + q, i0 + rows - 1);
#pragma unroll
    for (int dd = 0; dd < DIM; ++dd) {
      xf[q][dd] = d.x[(int64_t)i * DIM + dd];
      xq[q][dd] = (Real)xf[q][dd];
    }
  }
  const int nkc = (K + kFoldKC - 1) / kFoldKC;
  auto Y = [&](int kk, int dd, int t) -> float& { return ys[(kk * DIM + dd) * kFoldJC + t]; };
  auto stage = [&](int kc, int j0) {
    const int kb = kc * kFoldKC, nk = min(kFoldKC, K - kb);
    for (int e = threadIdx.x; e < nk * kFoldJC; e += blockDim.x) {
      const int kk = e / kFoldJC, t = e - kk * kFoldJC, jj = j0 + t;
#pragma unroll
      for (int dd = 0; dd < DIM; ++dd)
        Y(kk, dd, t) = jj < m ? d.y[((int64_t)(kb + kk) * m + jj) * DIM + dd] : 0.0f;
    }
  };
  for (int j0 = 0; j0 < m; j0 += kFoldJC) {
    const int j = j0 + tj;
    const bool active = grp_active && j < m;
    // pass 1 (float32): the shift, the minimum cost up to float32 rounding -- any shift that
    // close to the minimum keeps every shifted exponent <= ~0, and the same value is added
    // back exactly
    float cminf[kFoldQ];
#pragma unroll
    for (int q = 0; q < kFoldQ; ++q) cminf[q] = 3.0e38f;
    for (int kc = 0; kc < nkc; ++kc) {
      __syncthreads();  // the previous staging's readers are done
      stage(kc, j0);
      __syncthreads();
      const int nk = min(kFoldKC, K - kc * kFoldKC);
      if (active) {
#pragma unroll 4
        for (int kk = 0; kk < nk; ++kk) {
          float yv[DIM];
#pragma unroll
          for (int dd = 0; dd < DIM; ++dd) yv[dd] = Y(kk, dd, tj);
#pragma unroll
          for (int q = 0; q < kFoldQ; ++q) {
            float c = 0.0f;
#pragma unroll
            for (int dd = 0; dd < DIM; ++dd) { const float df = xf[q][dd] - yv[dd]; c = fmaf(df, df, c); }
            cminf[q] = fminf(c, cminf[q]);
          }
        }
      }
    }
    Real cmin[kFoldQ];
#pragma unroll
    for (int q = 0; q < kFoldQ; ++q) cmin[q] = (Real)cminf[q];
    float sum[kFoldQ] = {};
    for (int kc = 0; kc < nkc; ++kc) {
      if (nkc > 1) {
        __syncthreads();
        stage(kc, j0);
        __syncthreads();
      }
      const int nk = min(kFoldKC, K - kc * kFoldKC);
      if (active) {
#pragma unroll 4
        for (int kk = 0; kk < nk; ++kk) {
          Real yv[DIM];
#pragma unroll
          for (int dd = 0; dd < DIM; ++dd) yv[dd] = (Real)Y(kk, dd, tj);
#pragma unroll
          for (int q = 0; q < kFoldQ; ++q) {
            Real c = 0;
#pragma unroll
            for (int dd = 0; dd < DIM; ++dd) { const Real df = xq[q][dd] - yv[dd]; c = fma(df, df, c); }
            sum[q] += exp2_fast((float)((cmin[q] - c) * s2));
          }
        }
      }
    }
    if (active) {
      float v[kFoldQ];
#pragma unroll
      for (int q = 0; q < kFoldQ; ++q) v[q] = (float)(-cmin[q] * s2 + (Real)log2_fast(sum[q]));
#pragma unroll
      for (int q = 0; q < kFoldQ; ++q)
        if (ib + q < i0 + rows) L[(size_t)(ib + q) * mp + j] = v[q];
      float* lt = LT + (size_t)j * mp + ib;  // ib is a multiple of 4 and mp too: 16-byte aligned
      if (ib + kFoldQ <= i0 + rows) {
        *reinterpret_cast<float4*>(lt) = make_float4(v[0], v[1], v[2], v[3]);
      } else {
        for (int q = 0; q < kFoldQ && ib + q < i0 + rows; ++q) lt[q] = v[q];
      }
    }
  }
}

template <int DIM>
__device__ void fold_tile(const ot_batch_desc& d, int i0, int fp64_mode) {
  const int m = bm(d), K = d.K, mp = bmp(m);
  float* L = d.logK;
  float* LT = L + (size_t)m * mp;
  const int rows = min(kBT, m - i0);
  __shared__ float ys[kFoldKC * DIM * kFoldJC];
  if (fp64_mode != 0) fold_cols<DIM, double>(d, i0, rows, L, LT, ys);
  else fold_cols<DIM, float>(d, i0, rows, L, LT, ys);
  // padding: -inf contributes nothing to a log-sum-exp
  for (int e = threadIdx.x; e < rows * (mp - m); e += blockDim.x) {
    const int i = i0 + e / (mp - m), j = m + e % (mp - m);
    L[(size_t)i * mp + j] = -INFINITY;
  }
  // padding columns of the transpose (rows j < m, columns i in [m, mp)) are written by the
  // first tile
  if (i0 == 0) {
    for (int e = threadIdx.x; e < m * (mp - m); e += blockDim.x) {
      const int j = e / (mp - m), i = m + e % (mp - m);
      LT[(size_t)j * mp + i] = -INFINITY;
    }
  }
  if (i0 == 0) {  // exchange slots of a gang solve: epochs start at 1, so zero means "none"
    uint32_t* sw = reinterpret_cast<uint32_t*>(LT + (size_t)m * mp + 2 * (size_t)m);
    for (int e = threadIdx.x; e < 2 * (2 * mp + 2 * kMaxGangF); e += blockDim.x) sw[e] = 0u;
  }
  if (i0 == 0) {  // folded marginals
    float* al = LT + (size_t)m * mp;
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
// LSE2 of (row[j] + vec[j]) over j < mp by a group of LPR lanes in ONE pass: each lane keeps
// a running (max, sum) over its elements (four float4 per step, one rescale per step), then
// the group merges the pairs.  Rows and vec are 16-byte aligned and padded with -inf / 0 up
// to mp (a multiple of 4).  Every lane of the group returns the result.
template <int LPR>
__device__ __forceinline__ void grp_merge(float& M, float& S) {
  float m2 = dpp_f32<kDppXor1>(M), s2 = dpp_f32<kDppXor1>(S);
  lse_merge(M, S, m2, s2);
  m2 = dpp_f32<kDppXor2>(M); s2 = dpp_f32<kDppXor2>(S);
  lse_merge(M, S, m2, s2);
  m2 = dpp_f32<kDppHalfMirror>(M); s2 = dpp_f32<kDppHalfMirror>(S);
  lse_merge(M, S, m2, s2);
  m2 = dpp_f32<kDppMirror>(M); s2 = dpp_f32<kDppMirror>(S);
  lse_merge(M, S, m2, s2);
  if constexpr (LPR >= 32) {
    m2 = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(M), 0x401F));
    s2 = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(S), 0x401F));
    lse_merge(M, S, m2, s2);
  }
  if constexpr (LPR == 64) {
    m2 = __shfl_xor(M, 32, kWave);
    s2 = __shfl_xor(S, 32, kWave);
    lse_merge(M, S, m2, s2);
  }
}

template <int LPR>
__device__ __forceinline__ float grp_lse2(const float* row, const float* vec, int mp, int gl) {
  float M = kNegBig, S = 0.0f;
  for (int q = 4 * gl; q < mp; q += 16 * LPR) {
    float t[16];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int qq = q + 4 * LPR * u;
      if (qq < mp) {
        const float4 l = *reinterpret_cast<const float4*>(row + qq);
        const float4 v = *reinterpret_cast<const float4*>(vec + qq);
        t[4 * u] = l.x + v.x; t[4 * u + 1] = l.y + v.y; t[4 * u + 2] = l.z + v.z; t[4 * u + 3] = l.w + v.w;
      } else {
        t[4 * u] = t[4 * u + 1] = t[4 * u + 2] = t[4 * u + 3] = -INFINITY;
      }
    }
    float tm = t[0];
#pragma unroll
    for (int k = 1; k < 16; ++k) tm = fmaxf(tm, t[k]);
    const float Mn = fmaxf(M, tm);
    float acc = S * exp2_fast(M - Mn);
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += exp2_fast(t[k] - Mn);
    S = acc;
    M = Mn;
  }
  grp_merge<LPR>(M, S);
  return M + log2_fast(S);
}

constexpr float kMinShiftedSumB = 0x1p-60f;  // below this a shifted sum is redone exactly

// Shifted sum of 2^(row_j + vec_j + sh) over j < mp by a group of LPR lanes (rows padded
// with -inf); with sh the row's previous potential no maximum is needed (see the reduced
// solver).  Every lane of the group returns it.
template <int LPR>
__device__ __forceinline__ float grp_shifted_sum(const float* row, const float* vec, int mp,
                                                 int gl, float sh) {
  constexpr int kU = 4;  // loads in flight per lane (rows may stream from global memory)
  float s = 0.0f;
  for (int base = 4 * gl; base < mp; base += 4 * LPR * kU) {
    float4 l[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int q = base + 4 * LPR * u;
      l[u] = q < mp ? *reinterpret_cast<const float4*>(row + q)
                    : make_float4(-INFINITY, -INFINITY, -INFINITY, -INFINITY);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int q = base + 4 * LPR * u;
      if (q < mp) {
        const float4 v = *reinterpret_cast<const float4*>(vec + q);
        s += exp2_fast(l[u].x + (v.x + sh)) + exp2_fast(l[u].y + (v.y + sh)) +
             exp2_fast(l[u].z + (v.z + sh)) + exp2_fast(l[u].w + (v.w + sh));
      }
    }
  }
  s += dpp_f32<kDppXor1>(s);
  s += dpp_f32<kDppXor2>(s);
  s += dpp_f32<kDppHalfMirror>(s);
  s += dpp_f32<kDppMirror>(s);
  if constexpr (LPR >= 32) s = swap_sum16(s);
  if constexpr (LPR == 64) s = swap_sum32(s);
  return s;
}

struct BSolveArgs {
  const ot_batch_desc* descs;
  int count;
  const int32_t* ntasks;  // device: number of tasks (plan entry 3)
  const uint32_t* tasks;  // work queue, largest problems first: problem | member << 20 | (G-1) << 26
  uint32_t* queue;        // [0] next position, [1] abort flag; zeroed before the launch
  double tol;
  int max_iter;
  int warm;
};

template <int LPR>
__device__ void solve_one(const ot_batch_desc& d, const BSolveArgs& a, float* lds,
                          size_t lds_floats, float* red) {
  const int m = bm(d), K = d.K, mp = bmp(m);
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int gl = lane % LPR, grp = tid / LPR, ngrp = kBSolveThreads / LPR;
  // LDS: F, Fprev, G (mp each, zero padded), la2, lb2, al (m each) [+ L, LT when they fit]
  float* F = lds;
  float* Fp = F + mp;
  float* G = Fp + mp;
  float* la2 = G + mp;
  float* lb2 = la2 + mp;
  float* al = lb2 + mp;
  float* gL = d.logK;
  float* gLT = gL + (size_t)m * mp;
  const float* galpha = gLT + (size_t)m * mp;
  const float* gbeta = galpha + m;
  const bool in_lds = (size_t)6 * mp + (size_t)2 * m * mp <= lds_floats;
  const float* L = gL;
  const float* LT = gLT;
  if (in_lds) {
    float* Ls = al + mp;
    float* LTs = Ls + (size_t)m * mp;
    for (int e = tid; e < m * mp; e += blockDim.x) { Ls[e] = gL[e]; LTs[e] = gLT[e]; }
    L = Ls;
    LT = LTs;
  }
  for (int i = m + tid; i < mp; i += blockDim.x) { F[i] = 0.0f; G[i] = 0.0f; }
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
      const float Fo = F[i];
      float Fn, S = -1.0f;
      if (t >= 2) {  // shifted by the row's previous potential; exact when out of range
        S = grp_shifted_sum<LPR>(L + (size_t)i * mp, G, mp, gl, Fo);
        if (S >= kMinShiftedSumB && S < INFINITY) Fn = la2[i] - log2_fast(S) + Fo;
        else S = -1.0f;
      }
      if (S < 0.0f) Fn = la2[i] - grp_lse2<LPR>(L + (size_t)i * mp, G, mp, gl);
      if (gl == 0) {
        if (t >= 2) {
          // residual of the state after t-1: its row sum (the shifted sum) minus alpha
          const float rr = S >= 0.0f ? S - al[i] : scaled_exp2m1(al[i], Fo - Fn);
          racc += rr * rr;
        }
        Fp[i] = Fo;
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
      const float Go = G[j];
      const float S = grp_shifted_sum<LPR>(LT + (size_t)j * mp, F, mp, gl, Go);
      const float Gn = (S >= kMinShiftedSumB && S < INFINITY)
                           ? lb2[j] - log2_fast(S) + Go
                           : lb2[j] - grp_lse2<LPR>(LT + (size_t)j * mp, F, mp, gl);
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

// Exchange area of a problem's scratch, after its folded kernel, transpose and marginals:
// F and G slots (mp each) and residual-partial slots (2 x kMaxGang), 64-bit each.
constexpr int kMaxGang = kMaxGangF;
__device__ __forceinline__ uint64_t* gang_slots(const ot_batch_desc& d) {
  const int m = bm(d), mp = bmp(m);
  return reinterpret_cast<uint64_t*>(d.logK + 2 * (size_t)m * mp + 2 * (size_t)m);
}

// Shifted sum over j < mp of 2^(row_j + vec_j + sh) by one wave (rows padded with -inf up to
// mp, a multiple of 4); every lane returns it.  See the reduced solver for why no maximum is
// needed when sh is the row's previous potential.
// The row streams from global memory (L2 / MALL): eight float4 loads per lane are issued
// before any is used, so a wave keeps 8 KB in flight instead of waiting once per float4.
__device__ __forceinline__ float wave_shifted_sum_g(const float* __restrict__ row,
                                                    const float* __restrict__ vec, int mp,
                                                    int lane, float sh) {
  constexpr int kU = 8;
  float s = 0.0f;
  for (int base = 4 * lane; base < mp; base += 4 * kWave * kU) {
    float4 l[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int q = base + 4 * kWave * u;
      l[u] = q < mp ? *reinterpret_cast<const float4*>(row + q)
                    : make_float4(-INFINITY, -INFINITY, -INFINITY, -INFINITY);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int q = base + 4 * kWave * u;
      if (q < mp) {
        const float4 v = *reinterpret_cast<const float4*>(vec + q);
        s += exp2_fast(l[u].x + (v.x + sh)) + exp2_fast(l[u].y + (v.y + sh)) +
             exp2_fast(l[u].z + (v.z + sh)) + exp2_fast(l[u].w + (v.w + sh));
      }
    }
  }
  return wave_sum_v(s);
}


// One potential update of row (or column) `row` by one wave: lm - LSE2_j(row_j + vec_j),
// shifted by the previous potential when `shifted`, exact otherwise or when the shifted sum
// is out of range.  *S receives the previous plan's marginal sum, or -1 when not available.
__device__ __forceinline__ float gang_update(const float* row, const float* vec, int mp,
                                             int lane, float lm, float prev, bool shifted,
                                             float* S) {
  if (shifted) {
    const float s = wave_shifted_sum_g(row, vec, mp, lane, prev);
    if (s >= kMinShiftedSumB && s < INFINITY) {
      *S = s;
      return lm - log2_fast(s) + prev;
    }
  }
  *S = -1.0f;
  return lm - grp_lse2<64>(row, vec, mp, lane);
}

// A large problem solved by a gang of G workgroups (member k owns rows and columns
// [k R, k R + R), R = ceil(m / G)); the rows of the folded kernel stream from the scratch in
// global memory.  Same iteration, exchange and lagged stop test as the single-problem reduced
// solver: potentials and residual partials travel in epoch-tagged slots (agent scope; the
// members may sit on any XCD), two barriers per iteration, every member takes the same stop
// decision from the same partials.
__device__ void solve_gang(const ot_batch_desc& d, const BSolveArgs& a, int member, int G,
                           float* lds, uint32_t* abort_flag) {
  const int m = bm(d), K = d.K, mp = bmp(m);
  const int R = (m + G - 1) / G;
  const int r0 = member * R;
  const int nr = max(0, min(R, m - r0));
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const float* gL = d.logK;
  const float* gLT = gL + (size_t)m * mp;
  const float* galpha = gLT + (size_t)m * mp;
  const float* gbeta = galpha + m;
  uint64_t* fx = gang_slots(d);
  uint64_t* gx = fx + mp;
  uint64_t* rsx = gx + mp;  // [2][kMaxGang]
  float* VsG = lds;                 // [mp]
  float* VsF = VsG + mp;            // [mp]
  float* la2 = VsF + mp;            // [R] own rows / columns
  float* lb2 = la2 + R;
  float* av = lb2 + R;
  float* Fcur = av + R;
  float* Fprev = Fcur + R;
  float* Fold = Fprev + R;
  float* Gcur = Fold + R;
  float* Gprev = Gcur + R;
  float* rsv = Gprev + R;           // [kMaxGang]
  float* wsum = rsv + kMaxGang;     // [kBSolveWaves]
  int* flag = reinterpret_cast<int*>(wsum + kBSolveWaves);  // [0] s_bad
  const float s2 = (float)(kLog2eD / d.eps);
  for (int rl = tid; rl < R; rl += blockDim.x) {
    const bool ok = rl < nr;
    la2[rl] = ok ? log2f(galpha[r0 + rl]) : 0.0f;
    lb2[rl] = ok ? log2f(gbeta[r0 + rl]) : 0.0f;
    av[rl] = ok ? galpha[r0 + rl] : 0.0f;
    Gcur[rl] = ok && a.warm ? d.g[r0 + rl] * s2 : 0.0f;
    Gprev[rl] = Gcur[rl];
    Fcur[rl] = Fprev[rl] = Fold[rl] = 0.0f;
  }
  for (int j = tid; j < mp; j += blockDim.x) {
    VsG[j] = (j < m && a.warm) ? d.g[j] * s2 : 0.0f;
    VsF[j] = 0.0f;
  }
  if (tid == 0) flag[0] = 0;
  __syncthreads();
  const double tol2 = a.tol * a.tol / (double)K;
  int iters_done = 0, converged = 0, flags = 0;
  for (uint32_t t = 1;; ++t) {
    float racc = 0.0f;
    for (int rl = wv; rl < nr; rl += kBSolveWaves) {
      float S;
      const float Fo = Fcur[rl];
      const float Fn = gang_update(gL + (size_t)(r0 + rl) * mp, VsG, mp, lane, la2[rl], Fo,
                                   t >= 2, &S);
      if (lane == 0) {
        if (t >= 2) {
          const float rr = S >= 0.0f ? S - av[rl] : scaled_exp2m1(av[rl], Fo - Fn);
          racc += rr * rr;
        }
        Fold[rl] = Fprev[rl];
        Fprev[rl] = Fo;
        Fcur[rl] = Fn;
        slot_publish(fx + r0 + rl, Fn, t);
      }
    }
    if (lane == 0) wsum[wv] = racc;
    if (t >= 3) {  // stop test on the state after t-2, the same in every wave and member
      float sres = 0.0f;
      for (int v = lane; v < G; v += kWave) sres += rsv[v];
      sres = wave_sum_v(sres);
      const bool fin = sres == sres && sres < 3.0e38f;
      converged = fin && (double)sres <= tol2;
      if (!fin) flags |= 1;
      if ((converged && tol2 > 0.0) || !fin || (int)(t - 2) >= a.max_iter) {
        iters_done = (int)t - 2;
        break;
      }
    }
    if (!stage_slots(fx, m, mp, t, VsF, nullptr, 0, 0, nullptr, abort_flag, flag)) {
      flags |= 2;
      break;
    }
    if (wv == 0 && t >= 2) {
      float sw = lane < kBSolveWaves ? wsum[lane] : 0.0f;
      sw = wave_sum_v(sw);
      if (lane == 0) slot_publish(rsx + (t & 1u) * kMaxGang + member, sw, t);
    }
    for (int cl = wv; cl < nr; cl += kBSolveWaves) {
      float S;
      const float Go = Gcur[cl];
      const float Gn = gang_update(gLT + (size_t)(r0 + cl) * mp, VsF, mp, lane, lb2[cl], Go,
                                   true, &S);
      if (lane == 0) {
        Gprev[cl] = Go;
        Gcur[cl] = Gn;
        slot_publish(gx + r0 + cl, Gn, t);
      }
    }
    const int nres = t >= 2 ? G : 0;
    if (!stage_slots(gx, m, mp, t, VsG, rsx + (t & 1u) * kMaxGang, nres, t, rsv, abort_flag,
                     flag)) {
      flags |= 2;
      break;
    }
  }
  // outputs: the state after iteration iters_done, (F^{t-2}, G^{t-2}) as in the reduced solver
  __syncthreads();
  const float to_nat = (float)(d.eps * kLn2D);
  for (int rl = tid; rl < nr; rl += blockDim.x) {
    d.f[r0 + rl] = Fold[rl] * to_nat;
    d.g[r0 + rl] = Gprev[rl] * to_nat;
  }
  if (tid == 0 && (member == 0 || flags)) {
    if (member == 0) {
      d.out[5] = (double)iters_done;
      d.out[6] = (double)converged;
    }
    if (member == 0 || flags) d.out[7] = (double)flags;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kBSolveThreads) batched_solve_kernel(BSolveArgs a) {
  extern __shared__ float4 lds4[];
  float* lds = reinterpret_cast<float*>(lds4);
  __shared__ float red[kBSolveWaves];
  __shared__ uint32_t s_task;
  const size_t lds_floats = (size_t)kBMaxLds / sizeof(float);
  for (;;) {
    if (threadIdx.x == 0) {
      const uint32_t pos = __hip_atomic_fetch_add(a.queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_task = pos < (uint32_t)*a.ntasks ? a.tasks[pos] : 0xffffffffu;
    }
    __syncthreads();
    const uint32_t task = s_task;
    __syncthreads();
    if (task == 0xffffffffu) return;  // queue drained: every workgroup reaches this
    const int p = (int)(task & 0xfffffu);
    const int member = (int)((task >> 20) & 63u);
    const int G = (int)(task >> 26) + 1;
    const ot_batch_desc d = a.descs[p];
    if (G > 1) {
      solve_gang(d, a, member, G, lds, a.queue + 1);
      continue;
    }
    const int m = bm(d);
    const int lpr = d.tile_cfg == 16 || d.tile_cfg == 32 || d.tile_cfg == 64
                        ? d.tile_cfg : (m >= 512 ? 64 : m >= 128 ? 32 : 16);
    if (lpr == 64) solve_one<64>(d, a, lds, lds_floats, red);
    else if (lpr == 32) solve_one<32>(d, a, lds, lds_floats, red);
    else solve_one<16>(d, a, lds, lds_floats, red);
  }
}

// ---- 3. values, gradients and float64 marginal sums ----------------------------------------
// Tiles [0, nrow) of a problem are row tiles, [nrow, 2 nrow) column tiles (16 points each: a
// wave owns 4 points and its lanes stride over the partner points, so one partner load feeds
// four entries).
// acc[p]: {P, <C,T>, mass, sum (rowsum - alpha)^2, sum (colsum - beta)^2, <f,alpha>, <g,beta>}
constexpr int kVChunk = 1024;  // partner points staged in LDS at a time (4 per thread)

template <int DIM, bool ROW>
__device__ void values_tile(const ot_batch_desc& d, int a0, double* __restrict__ acc,
                           float4* __restrict__ sP, float4* __restrict__ sC) {
  constexpr int Q = 4;
  const int m = bm(d), K = d.K, mp = bmp(m);
  const float* L = d.logK;
  const float* LT = L + (size_t)m * mp;
  const float* al = LT + (size_t)m * mp;
  const float* be = al + m;
  const float s2 = (float)(kLog2eD / d.eps);
  const double s2d = kLog2eD / d.eps;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int A0 = a0 + wv * Q;  // first own point of this wave (row i or column j)
  const bool active = A0 < m;  // inactive waves still stage partners and meet the barriers
  const float* ownp = ROW ? d.x : d.y;
  const float* othp = ROW ? d.y : d.x;
  int Aq[Q];
  float po[Q][DIM], pa[Q], gacc[Q][DIM], tP[Q], tC[Q], tM[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    Aq[q] = min(A0 + q, m - 1);
#pragma unroll
    for (int dd = 0; dd < DIM; ++dd) { po[q][dd] = ownp[(int64_t)Aq[q] * DIM + dd]; gacc[q][dd] = 0.0f; }
    pa[q] = ROW ? d.f[Aq[q]] : d.g[Aq[q]];
    tP[q] = tC[q] = tM[q] = 0.0f;
  }
  // Partner points b of a chunk are staged in LDS: sC[b] = {cost point, partner potential}
  // once per chunk (ROW: nothing but g_b; COL: x_b of block-row 0 and f_b), sP[b] = the
  // gradient partner of block k (ROW: y_{k m + b}; COL: x_{r m + b}, r = (K - k) mod K, whose
  // entry with column j is T_{b j k}).
  // potentials enter the exponent scaled to base 2: pas (own) and sC.w (partner)
  float pas[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) pas[q] = pa[q] * s2;
  constexpr int kPre = kVChunk / 256;  // partners per thread per block (256 threads)
  for (int c0 = 0; c0 < m; c0 += kVChunk) {
    const int nc = min(kVChunk, m - c0);
    __syncthreads();  // the previous chunk's readers are done
    for (int b = threadIdx.x; b < nc; b += blockDim.x) {
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (!ROW) {
        v.x = d.x[(int64_t)(c0 + b) * DIM];
        v.y = d.x[(int64_t)(c0 + b) * DIM + 1];
        if (DIM == 3) v.z = d.x[(int64_t)(c0 + b) * DIM + 2];
      }
      v.w = (ROW ? d.g[c0 + b] : d.f[c0 + b]) * s2;
      sC[b] = v;
    }
    // the partners of block k + 1 are loaded into registers while block k is processed
    float4 pre[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int b = threadIdx.x + 256 * u;
      const int64_t P = (int64_t)c0 + b;  // block 0 (k = 0, r = 0)
      pre[u] = b < nc ? make_float4(othp[P * DIM], othp[P * DIM + 1], DIM == 3 ? othp[P * DIM + 2] : 0.f, 0.f)
                      : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    for (int k = 0; k < K; ++k) {
      __syncthreads();  // sP of the previous block is no longer read
#pragma unroll
      for (int u = 0; u < kPre; ++u) {
        const int b = threadIdx.x + 256 * u;
        if (b < nc) sP[b] = pre[u];
      }
      __syncthreads();
      if (k + 1 < K) {
        const int kn = k + 1, rn = (K - kn) % K;
        const int64_t pbase = (int64_t)(ROW ? kn : rn) * m + c0;
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
          const int b = threadIdx.x + 256 * u;
          const int64_t P = pbase + b;
          if (b < nc)
            pre[u] = make_float4(othp[P * DIM], othp[P * DIM + 1], DIM == 3 ? othp[P * DIM + 2] : 0.f, 0.f);
        }
      }
      if (!active) continue;
      float yk[Q][DIM];  // COL: y_{k m + j} of the own columns j
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int dd = 0; dd < DIM; ++dd) yk[q][dd] = ROW ? 0.0f : d.y[(int64_t)(k * m + Aq[q]) * DIM + dd];
      for (int b = lane; b < nc; b += kWave) {
        const float4 P4 = sP[b];
        const float4 C4 = sC[b];
        const float pp[3] = {P4.x, P4.y, P4.z};
        // ROW: the cost uses the partner itself; COL: block-row 0's row point x_b
        const float cb[3] = {ROW ? P4.x : C4.x, ROW ? P4.y : C4.y, ROW ? P4.z : C4.z};
        const float obs = C4.w;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          float c = 0.0f;
#pragma unroll
          for (int dd = 0; dd < DIM; ++dd) {
            // ROW: C_{i, b, k} = |x_i - y_{k m + b}|^2; COL: C_{b, j, k} = |x_b - y_{k m + j}|^2
            const float df = ROW ? po[q][dd] - cb[dd] : cb[dd] - yk[q][dd];
            c = fmaf(df, df, c);
          }
          const float T = exp2_fast(fmaf(-c, s2, pas[q] + obs));
#pragma unroll
          for (int dd = 0; dd < DIM; ++dd) gacc[q][dd] = fmaf(T, po[q][dd] - pp[dd], gacc[q][dd]);
          if (ROW) {
            // C + eps (Z - 1) = f_i + g_j - eps with Z = (f_i + g_j - C) / eps: the primal
            // term needs only the plan's g-weighted sum (kept scaled by s2) besides its mass
            tP[q] = fmaf(T, obs, tP[q]);
            tC[q] = fmaf(T, c, tC[q]);
            tM[q] += T;
          }
        }
      }
    }
  }
  if (!active) return;
  double vP = 0.0, vC = 0.0, vM = 0.0, v2 = 0.0, vd = 0.0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const bool ok = A0 + q < m;
    // marginal sum of the own point from logK (base 2 in the scratch): float64 exponents and
    // sums, float32 exponentials of the exponents less the own potential's part, scaled back
    // exactly (the terms of a converged row are at most the row's marginal, far from
    // under- or overflow after the shift)
    const float* Lrow = (ROW ? L : LT) + (size_t)Aq[q] * mp;
    const double own2 = (double)pa[q] * s2d;
    const float* opot = ROW ? d.g : d.f;
    float emax = -INFINITY;
    for (int b = lane; b < m; b += kWave)
      emax = fmaxf(emax, (float)((double)Lrow[b] + (double)opot[b] * s2d + own2));
    const double sh2 = (double)wave_max_v(emax);
    double ms = 0.0;
    for (int b = lane; b < m; b += kWave)
      ms += (double)exp2_fast((float)((double)Lrow[b] + (double)opot[b] * s2d + own2 - sh2));
    ms = wave_sum_d(ms) * exp2(sh2);
    const double target = ROW ? (double)al[Aq[q]] : (double)be[Aq[q]];
#pragma unroll
    for (int dd = 0; dd < DIM; ++dd) {
      const float gsum = wave_sum(gacc[q][dd]);
      float* dst = ROW ? d.dx : d.dy;
      if (lane == 0 && dst && ok) dst[(int64_t)Aq[q] * DIM + dd] = 2.0f * gsum;
    }
    if (ROW) {
      const double Tg = wave_sum_d((double)tP[q]) / (double)s2, C = wave_sum_d((double)tC[q]),
                   Ms = wave_sum_d((double)tM[q]);
      // sum_{j,k} T_ijk (f_i + g_j - eps)
      if (ok) { vP += ((double)pa[q] - d.eps) * Ms + Tg; vC += C; vM += Ms; }
    }
    if (ok) {
      v2 += (ms - target) * (ms - target);
      vd += (double)pa[q] * target;
    }
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
  __shared__ float4 sP[kVChunk], sC[kVChunk];
  if (d.dim == 3) { if (row) values_tile<3, true>(d, a0, acc, sP, sC); else values_tile<3, false>(d, a0, acc, sP, sC); }
  else { if (row) values_tile<2, true>(d, a0, acc, sP, sC); else values_tile<2, false>(d, a0, acc, sP, sC); }
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

size_t batched_plan_len(int count) { return 4 + (3 + (size_t)kMaxGangF) * (size_t)count; }

// Workgroups that solve one problem together: one up to m = 256 (logK then costs a single
// workgroup at most ~0.1 ms per solve), about 128 rows per member above.
static int gang_size(int m) {
  if (m <= 256) return 1;
  const int g = (m + 127) / 128;
  return g < kMaxGangF ? g : kMaxGangF;
}

// plan = {nfold, nval, count, ntasks, order[count], fold_start[count], val_start[count],
//         tasks[ntasks]}; a task is problem | member << 20 | (G - 1) << 26, largest problems
// first, the G members of a gang consecutive.
int batched_plan(const ot_batch_desc* h, int count, int32_t* plan) {
  if (count >= (1 << 20)) return -1;
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
  uint32_t* tasks = reinterpret_cast<uint32_t*>(vstart + count);
  int64_t nf = 0, nv = 0;
  int nt = 0;
  for (int p = 0; p < count; ++p) {
    order[p] = idx[p];
    const int m = h[p].n / h[p].K;
    const int tiles = (m + kBT - 1) / kBT;
    fstart[p] = (int32_t)nf;
    vstart[p] = (int32_t)nv;
    nf += tiles;
    nv += 2 * tiles;
  }
  for (int q = 0; q < count; ++q) {
    const int p = idx[q];
    const int G = gang_size(h[p].n / h[p].K);
    for (int k = 0; k < G; ++k) tasks[nt++] = (uint32_t)p | ((uint32_t)k << 20) | ((uint32_t)(G - 1) << 26);
  }
  if (nf > INT32_MAX || nv > INT32_MAX) return -1;
  plan[0] = (int32_t)nf;
  plan[1] = (int32_t)nv;
  plan[2] = count;
  plan[3] = nt;
  return 0;
}

size_t batched_ws_bytes(int count) { return a256(256) + a256(sizeof(double) * 8 * (size_t)count); }

hipError_t launch_batched(const ot_batch_desc* descs, int count, const int32_t* dplan,
                          int nfold, int nval, double tol, int max_iter, int fold_fp64,
                          int warm, void* ws, hipStream_t s, hipEvent_t* events) {
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
  // the device copy of the plan: task count in entry 3, tasks after val_start
  const uint32_t* tasks = reinterpret_cast<const uint32_t*>(vstart + count);
  BSolveArgs a{descs, count, dplan + 3, tasks, queue, tol, max_iter, warm};
  // one workgroup per CU (the LDS request allows no more), all resident at once, so the
  // members of a gang never wait on a workgroup that cannot start; workgroups that find the
  // queue empty leave at once
  const int grid = cus;
  if (events && (e = hipEventRecord(events[0], s)) != hipSuccess) return e;
  hipLaunchKernelGGL(batched_solve_kernel, dim3(grid), dim3(kBSolveThreads), kBMaxLds, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (events && (e = hipEventRecord(events[1], s)) != hipSuccess) return e;
  hipLaunchKernelGGL(batched_values_kernel, dim3(nval), dim3(256), 0, s, descs, count, vstart, accs);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(batched_finalize_kernel, dim3((count + 255) / 256), dim3(256), 0, s, descs,
                     count, accs);
  return hipGetLastError();
}

}  // namespace csot
