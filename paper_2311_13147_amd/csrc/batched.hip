// Many independent reduced problems of uneven size in one stream of four launches, all
// capturable in a HIP graph (no host synchronisation, no memset, no allocation):
//
//   1. fold   : tiles of 32 rows of one problem -> logK (base 2) and its transpose, alpha, beta
//               (eq. def_Kij; Alg. 3 stage-1 averaging of the marginals);
//   2. solve  : ONE persistent launch; each workgroup pops the next problem from a device work
//               queue (largest first) and runs the cyclic Sinkhorn loop of Alg. 2 on it alone,
//               synchronising only within the workgroup; logK stays in LDS when it fits;
//   3. values : tiles of 4 rows (or columns) of block 0 of one problem, one wave per point ->
//               objective terms, marginal sums and the gradients of every point;
//   4. finalize per problem: P, D, <C,T>, errors.
//
// Per problem the cost is block-row 0's: C_ijk = |x_i - y_{k m + j}|^2.  The gradients are
// those of the full problem's objective with respect to all n points and both marginals (the
// envelope gradients of the single-problem ot_cost_and_grad):
//   dx_I = 2 sum_J T_IJ (x_I - y_J),  dy_J = 2 sum_I T_IJ (y_J - x_I),
//   da = f - mean(f), db = g - mean(g) (tiled),
// with T the expanded plan T[r m + i, c m + j] = T_{ij,(c-r) mod K} (Lemma 1).
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "launch.hpp"
#include "csot.h"

namespace csot {

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
// A tile is kFoldRows rows of one problem, kFoldQ of them per wave; a lane owns one column j of
// a 64-column chunk.  The rows of a wave are the same for all its lanes, so their terms a =
// 2 s2 x_i live in scalar registers and enter the vector FMAs as scalar operands, leaving the
// vector registers to the per-lane state (shift and sum of each row).  For each chunk the
// target points y_{k m + j} of up to kFoldKC shifts are staged in LDS (float32 coordinates
// and -s2 |y|^2 in float64, formed once per point); with K <= kFoldKC one staging serves both
// passes and the next chunk's points are fetched into registers while this one is computed.
// Each staged point serves the tile's kFoldRows rows.  Two passes over k: the shift, then
// the shifted exponential sum.  Output in base 2 (log2 of the folded kernel), in both layouts.
//
// fp64 (default): with s2 = log2(e) / eps, a = 2 s2 x_i (per row) and P = s2 |y|^2 (per
// staged point), u_k = a . y_k - P_k = s2 (|x_i|^2 - C_ijk) costs DIM float64 FMAs; pass 1
// takes U = max_k u_k, pass 2 sums 2^(u_k - U) (exponents formed in float64, exponentials in
// float32), and log2 K_ij = U - s2 |x_i|^2 + log2(sum).  Expanding the square cancels terms
// of size s2 (|x|^2 + |y|^2), which float64 carries with ~1e-16 relative rounding: the
// exponents stay exact far below float32's output rounding.  fp32 (fold_fp64 = 0): the
// squared differences directly in float32 (no cancellation beyond the cost's own rounding).
constexpr int kFoldQ = 8;                        // rows per wave
constexpr int kFoldThreads = 256;                // 4 waves
constexpr int kFoldRows = kFoldQ * kFoldThreads / kWave;  // rows per tile (32)
constexpr int kFoldJC = 64;                      // target columns j per staging (one per lane)
constexpr int kFoldKC = 32;                      // shifts k per staging
constexpr int kFoldSR = kFoldKC * kFoldJC / kFoldThreads;  // staged points per thread
constexpr int kFoldCB = 256;                     // columns per tile unless tile_cfg says

__host__ __device__ __forceinline__ int fold_row_blocks(int m) {
  return (m + kFoldRows - 1) / kFoldRows;
}
// columns per fold tile: tile_cfg bits 8-15 in units of 64, 0 = kFoldCB
__host__ __device__ __forceinline__ int fold_cb_width(int tile_cfg) {
  const int c = (tile_cfg >> 8) & 0xff;
  return c > 0 ? 64 * c : kFoldCB;
}
__host__ __device__ __forceinline__ int fold_col_blocks(int m, int tile_cfg) {
  const int w = fold_cb_width(tile_cfg);
  return (m + w - 1) / w;
}

template <int DIM>
struct FoldShared {
  float y[DIM * kFoldKC * kFoldJC];  // [DIM][kFoldKC][kFoldJC], as given
  double np[kFoldKC * kFoldJC];      // -s2 |y|^2
};

// max(a, b) of two float64 values by v_max_f64 alone: a running maximum through fmax is
// re-canonicalised (NaN-quieted) on every use, which costs a second instruction per term.
__device__ __forceinline__ double vmax_f64(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// A wave-uniform double moved to scalar registers.
__device__ __forceinline__ double uniform_d(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ void store_fold_row(float* L, float* LT, int mp, int i0, int rows,
                                               int ib, int j, const float (&v)[kFoldQ]) {
#pragma unroll
  for (int q = 0; q < kFoldQ; ++q)
    if (ib + q < i0 + rows) L[(size_t)(ib + q) * mp + j] = v[q];
  float* lt = LT + (size_t)j * mp + ib;  // ib is a multiple of 8 and mp of 4: 16-byte aligned
  if (ib + kFoldQ <= i0 + rows) {
#pragma unroll
    for (int q = 0; q < kFoldQ; q += 4)
      *reinterpret_cast<float4*>(lt + q) = make_float4(v[q], v[q + 1], v[q + 2], v[q + 3]);
  } else {
    for (int q = 0; q < kFoldQ && ib + q < i0 + rows; ++q) lt[q] = v[q];
  }
}

template <int DIM, bool F64>
__device__ void fold_tile(const ot_batch_desc& d, int rb, int cb, FoldShared<DIM>& sh) {
  const int m = bm(d), K = d.K, mp = bmp(m);
  const int cbw = fold_cb_width(d.tile_cfg);
  const int i0 = rb * kFoldRows, jb = cb * cbw, je = min(m, jb + cbw);
  float* L = d.logK;
  float* LT = L + (size_t)m * mp;
  const int rows = min(kFoldRows, m - i0);
  const double s2 = kLog2eD / d.eps;
  const float s2f = (float)s2;
  const int tj = threadIdx.x % kFoldJC, grp = threadIdx.x / kFoldJC;
  const int ib = i0 + grp * kFoldQ;
  const bool grp_active = ib < i0 + rows;  // inactive waves still stage and meet barriers
  // the wave's rows: a = 2 s2 x (float64, scalar registers) or x (float32)
  double ax[kFoldQ][DIM];
  float xf[kFoldQ][DIM];
#pragma unroll
  for (int q = 0; q < kFoldQ; ++q) {
    const int i = min(ib + q, i0 + rows - 1);
#pragma unroll
    for (int dd = 0; dd < DIM; ++dd) {
      xf[q][dd] = d.x[(int64_t)i * DIM + dd];
      ax[q][dd] = uniform_d(2.0 * s2 * (double)xf[q][dd]);
    }
  }
  const int nkc = (K + kFoldKC - 1) / kFoldKC;
  // staging in two steps: the global loads into registers, then the LDS stores
  float pre[kFoldSR][DIM];
  auto fetch = [&](int kc, int j0) {
    const int kb = kc * kFoldKC, nk = min(kFoldKC, K - kb);
#pragma unroll
    for (int r = 0; r < kFoldSR; ++r) {
      const int e = threadIdx.x + r * kFoldThreads, kk = e / kFoldJC, jj = j0 + e % kFoldJC;
#pragma unroll
      for (int dd = 0; dd < DIM; ++dd)
        pre[r][dd] = kk < nk && jj < m ? d.y[((int64_t)(kb + kk) * m + jj) * DIM + dd] : 0.0f;
    }
  };
  auto put = [&](int kc) {
    const int nk = min(kFoldKC, K - kc * kFoldKC);
#pragma unroll
    for (int r = 0; r < kFoldSR; ++r) {
      const int e = threadIdx.x + r * kFoldThreads, kk = e / kFoldJC, t = e % kFoldJC;
      if (kk < nk) {
        double n2 = 0.0;
#pragma unroll
        for (int dd = 0; dd < DIM; ++dd) {
          sh.y[(dd * kFoldKC + kk) * kFoldJC + t] = pre[r][dd];
          n2 = fma((double)pre[r][dd], (double)pre[r][dd], n2);
        }
        if constexpr (F64) sh.np[kk * kFoldJC + t] = -s2 * n2;
      }
    }
  };
  auto ld = [&](int kk, float (&yv)[DIM], double& np) {
#pragma unroll
    for (int dd = 0; dd < DIM; ++dd) yv[dd] = sh.y[(dd * kFoldKC + kk) * kFoldJC + tj];
    if constexpr (F64) np = sh.np[kk * kFoldJC + tj];
  };
  if (nkc == 1) fetch(0, jb);
  for (int j0 = jb; j0 < je; j0 += kFoldJC) {
    const int j = j0 + tj;
    const bool active = grp_active && j < je;
    double U[kFoldQ];
    float cminf[kFoldQ], sum[kFoldQ];
#pragma unroll
    for (int q = 0; q < kFoldQ; ++q) {
      U[q] = -INFINITY;
      cminf[q] = 3.0e38f;
      sum[q] = 0.0f;
    }
    // pass 1: the shift (F64: U = max_k u_k; fp32: the minimum cost)
    for (int kc = 0; kc < nkc; ++kc) {
      __syncthreads();  // the previous staging's readers are done
      if (nkc > 1) fetch(kc, j0);
      put(kc);
      __syncthreads();
      if (nkc == 1 && j0 + kFoldJC < je) fetch(0, j0 + kFoldJC);  // in flight during the passes
      const int nk = min(kFoldKC, K - kc * kFoldKC);
      if (active) {
#pragma unroll 2
        for (int kk = 0; kk < nk; ++kk) {
          float yv[DIM];
          double np = 0.0;
          ld(kk, yv, np);
          if constexpr (F64) {
            double yd[DIM];
#pragma unroll
            for (int dd = 0; dd < DIM; ++dd) yd[dd] = (double)yv[dd];
#pragma unroll
            for (int q = 0; q < kFoldQ; ++q) {
              double u = np;
#pragma unroll
              for (int dd = 0; dd < DIM; ++dd) u = fma(ax[q][dd], yd[dd], u);
              U[q] = vmax_f64(U[q], u);
            }
          } else {
#pragma unroll
            for (int q = 0; q < kFoldQ; ++q) {
              float c = 0.0f;
#pragma unroll
              for (int dd = 0; dd < DIM; ++dd) {
                const float df = xf[q][dd] - yv[dd];
                c = fmaf(df, df, c);
              }
              cminf[q] = fminf(c, cminf[q]);
            }
          }
        }
      }
    }
    // pass 2: the shifted exponential sum
    for (int kc = 0; kc < nkc; ++kc) {
      if (nkc > 1) {
        __syncthreads();
        fetch(kc, j0);
        put(kc);
        __syncthreads();
      }
      const int nk = min(kFoldKC, K - kc * kFoldKC);
      if (active) {
#pragma unroll 2
        for (int kk = 0; kk < nk; ++kk) {
          float yv[DIM];
          double np = 0.0;
          ld(kk, yv, np);
          if constexpr (F64) {
            double yd[DIM];
#pragma unroll
            for (int dd = 0; dd < DIM; ++dd) yd[dd] = (double)yv[dd];
#pragma unroll
            for (int q = 0; q < kFoldQ; ++q) {
              double u = np - U[q];
#pragma unroll
              for (int dd = 0; dd < DIM; ++dd) u = fma(ax[q][dd], yd[dd], u);
              sum[q] += exp2_fast((float)u);
            }
          } else {
#pragma unroll
            for (int q = 0; q < kFoldQ; ++q) {
              float c = 0.0f;
#pragma unroll
              for (int dd = 0; dd < DIM; ++dd) {
                const float df = xf[q][dd] - yv[dd];
                c = fmaf(df, df, c);
              }
              sum[q] += exp2_fast((cminf[q] - c) * s2f);
            }
          }
        }
      }
    }
    if (active) {
      float v[kFoldQ];
#pragma unroll
      for (int q = 0; q < kFoldQ; ++q) {
        if constexpr (F64) {
          double xx = 0.0;  // s2 |x|^2 = |a|^2 / (4 s2)
#pragma unroll
          for (int dd = 0; dd < DIM; ++dd) xx = fma(ax[q][dd], ax[q][dd], xx);
          v[q] = (float)((U[q] - xx / (4.0 * s2)) + (double)log2_fast(sum[q]));
        } else {
          v[q] = -cminf[q] * s2f + log2_fast(sum[q]);
        }
      }
      store_fold_row(L, LT, mp, i0, rows, ib, j, v);
    }
  }
  // padding: -inf contributes nothing to a log-sum-exp.  Columns [m, mp) of the tile's rows
  // (by the last column block), and of the transpose's rows j of the tile's columns (by the
  // first row block)
  if (cb == fold_col_blocks(m, d.tile_cfg) - 1) {
    for (int e = threadIdx.x; e < rows * (mp - m); e += blockDim.x) {
      const int i = i0 + e / (mp - m), j = m + e % (mp - m);
      L[(size_t)i * mp + j] = -INFINITY;
    }
  }
  if (rb == 0) {
    for (int e = threadIdx.x; e < (je - jb) * (mp - m); e += blockDim.x) {
      const int j = jb + e / (mp - m), i = m + e % (mp - m);
      LT[(size_t)j * mp + i] = -INFINITY;
    }
  }
  if (rb == 0 && cb == 0) {  // exchange slots of a gang solve: epochs start at 1 ("none" = 0)
    uint32_t* sw = reinterpret_cast<uint32_t*>(LT + (size_t)m * mp + 2 * (size_t)m);
    for (int e = threadIdx.x; e < 2 * (2 * mp + 2 * kMaxGangF); e += blockDim.x) sw[e] = 0u;
  }
  if (rb == 0 && cb == 0) {  // folded marginals
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

// Tiles in the solve order (the largest problems first, so that the small tiles fill the
// end of the launch); a tile is (row block, column block) of problem order[q].
template <bool F64>
__global__ void __launch_bounds__(kFoldThreads)
    batched_fold_kernel(const ot_batch_desc* __restrict__ descs, int count,
                        const int32_t* __restrict__ order, const int32_t* __restrict__ tile_start) {
  const int q = find_problem(tile_start, count, blockIdx.x);
  const ot_batch_desc d = descs[order[q]];
  const int m = bm(d), ncb = fold_col_blocks(m, d.tile_cfg);
  const int t = blockIdx.x - tile_start[q];
  if (t >= fold_row_blocks(m) * ncb) return;
  __shared__ FoldShared<3> sh;
  if (d.dim == 3) fold_tile<3, F64>(d, t / ncb, t % ncb, sh);
  else fold_tile<2, F64>(d, t / ncb, t % ncb, *reinterpret_cast<FoldShared<2>*>(&sh));
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
    const int cfg = d.tile_cfg & 0xff;
    const int lpr = cfg == 16 || cfg == 32 || cfg == 64 ? cfg : (m >= 512 ? 64 : m >= 128 ? 32 : 16);
    if (lpr == 64) solve_one<64>(d, a, lds, lds_floats, red);
    else if (lpr == 32) solve_one<32>(d, a, lds, lds_floats, red);
    else solve_one<16>(d, a, lds, lds_floats, red);
  }
}

// ---- 3. values and gradients of every point ------------------------------------------------
// Every plan entry T_ijk is evaluated once per pass, and the gradients of all K copies of an own
// point of block 0 come from float64 circular sums over the blocks:
//   row i   : Y(r) = sum_{k,j} T_ijk y_{((r + k) mod K) m + j},  dx_{r m + i} = 2 (x_{r m + i} S_i - Y(r));
//   column j: X(c) = sum_{k,i} T_ijk x_{((c - k) mod K) m + i},  dy_{c m + j} = 2 (y_{c m + j} S'_j - X(c)).
// For K in {1, 2, 4, 8, 16, 32} they run as a matrix product on the float64 matrix cores
// (bgrad_tile, 16 own points per wave); any other K takes badj_point: one wave per own point,
// four per workgroup (tiles [0, ceil(m / 4)) of a problem are row tiles, the next as many
// column tiles), lanes over the partners, one output block at a time with the plan entries
// re-evaluated per block.
// acc[p]: {P, <C,T>, mass, sum (rowsum - alpha)^2, sum (colsum - beta)^2, <f,alpha>, <g,beta>}
constexpr int kAdjPts = 4;  // own points (waves) per workgroup

constexpr int kAdjChunk = 64;  // partners staged in LDS at a time (one per lane)

// Generic K.  Called by all four waves of the workgroup; a wave whose own point lies beyond m
// passes active = false.
template <int DIM, bool ROW>
__device__ void badj_point(const ot_batch_desc& d, int o, bool active, int lane, double* vals) {
  const int m = bm(d), K = d.K;
  const float s2 = (float)(kLog2eD / d.eps);
  const float eps = (float)d.eps;
  gcfloat* x = as_global(d.x);
  gcfloat* y = as_global(d.y);
  gcfloat* fpot = as_global(d.f);
  gcfloat* gpot = as_global(d.g);
  float* __restrict__ gout = ROW ? d.dx : d.dy;
  const bool grad = gout != nullptr;
  const int oc = active ? o : 0;  // an inactive wave reads a valid point and writes nothing
  const float po = ROW ? fpot[oc] : gpot[oc];
  float xo[DIM];
  if constexpr (ROW) {
#pragma unroll
    for (int dd = 0; dd < DIM; ++dd) xo[dd] = x[oc * DIM + dd];
  }
  gcfloat* src = ROW ? y : x;   // the partner's copies in every block
  auto cost_T = [&](int p, int k, float fg, float& c) -> float {
    c = 0.0f;
#pragma unroll
    for (int dd = 0; dd < DIM; ++dd) {
      // |x_i - y_{k m + j}|^2: row pass partner j = p, column pass partner i = p
      const float e = ROW ? xo[dd] - y[(k * m + p) * DIM + dd]
                          : x[p * DIM + dd] - y[(k * m + o) * DIM + dd];
      c = fmaf(e, e, c);
    }
    return exp2_fast((fg - c) * s2);
  };
  double S = 0.0;
  float vP = 0.0f, vC = 0.0f;
  if (!active) return;
  // output block r at a time, the plan entries re-evaluated per block
#pragma unroll 1
  for (int r = 0; r < (grad ? K : 1); ++r) {
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int p = lane; p < m; p += kWave) {
      const float fg = po + (ROW ? gpot[p] : fpot[p]);
#pragma unroll 1
      for (int k = 0; k < K; ++k) {
        float c;
        const float T = cost_T(p, k, fg, c);
        if (r == 0) {
          S += (double)T;
          if (ROW) {
            vP = fmaf(T, fg - eps, vP);
            vC = fmaf(T, c, vC);
          }
        }
        if (grad) {
          const int a = ROW ? (r + k) % K : (r - k + K) % K;
#pragma unroll
          for (int dd = 0; dd < DIM; ++dd)
            a4[dd] = fma((double)T, (double)src[(a * m + p) * DIM + dd], a4[dd]);
        }
      }
    }
    if (r == 0) S = wave_sum_all_d(S);
    if (grad) {
#pragma unroll
      for (int dd = 0; dd < DIM; ++dd) {
        const double v = wave_sum_all_d(a4[dd]);
        const int P = r * m + o;
        if (lane == 0)
          gout[P * DIM + dd] = (float)(2.0 * ((double)(ROW ? x : y)[P * DIM + dd] * S - v));
      }
    }
  }
  // the folded marginal of the own point and the mean of its potential (da, db)
  double mv = 0.0, ps = 0.0;
  gcfloat* marg_in = as_global(ROW ? d.a : d.b);
  for (int r = lane; r < K; r += kWave) mv += (double)marg_in[r * m + o];
  gcfloat* pot = ROW ? fpot : gpot;
  for (int q = lane; q < m; q += kWave) ps += (double)pot[q];
  const double marg = wave_sum_all_d(mv) / K;
  const double pmean = wave_sum_all_d(ps) / m;
  float* __restrict__ dpot = ROW ? d.da : d.db;
  if (dpot)
    for (int r = lane; r < K; r += kWave) dpot[r * m + o] = (float)((double)po - pmean);
  const double tP = ROW ? wave_sum_all_d((double)vP) : 0.0;
  const double tC = ROW ? wave_sum_all_d((double)vC) : 0.0;
  if (lane == 0) {
    const double dr = S - marg;
    vals[0] = tP;
    vals[1] = tC;
    vals[2] = ROW ? S : 0.0;
    vals[3] = dr * dr;
    vals[4] = (double)po * marg;
  }
}

// ---- gradients on the float64 matrix cores (K in {1, 2, 4, 8, 16, 32}) --------------------
// For the K copies of an own point the circular sums above are one matrix product per pass:
//   row    : Y[i, (r, d)] = sum_{(k, j)} T_ijk B[(k, j), (r, d)],  B = y_{((r + k) mod K) m + j, d}
//   column : X[j, (c, d)] = sum_{(k, i)} T_ijk B[(k, i), (c, d)],  B = x_{((c - k) mod K) m + i, d}
// (inner index (shift, partner), K DIM output columns).  A wave takes 16 own points; for each
// quad of partners and each shift its 64 lanes evaluate the 16 x 4 plan entries T (lane l: own
// point l mod 16, partner l / 16) -- the A operand of v_mfma_f64_16x16x4f64 -- and gather the
// matching 4 x 16 B operands from the staged partner copies, one per tile of 16 output columns.
// Every plan entry is evaluated once per pass, and the float64 products and sums run on the
// matrix cores.  The lane layout: A[l mod 16][l / 16], B[l / 16][l mod 16], and the four
// results of lane l are D[l / 16 + 4 v][l mod 16], v = 0..3.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kMfPts = 16;                      // own points per wave
constexpr int kGradPts = kAdjPts * kMfPts;      // own points per gradient tile
constexpr int kGradChunk = 32;                  // partners staged in LDS at a time

// LDS geometry of a class: a staged partner holds its NC = K DIM copy components twice in a
// row (so that the component of block (r + k) mod K or (c - k) mod K is read at r DIM + d +
// k DIM or c DIM + d + NC - k DIM without a wrap), rows kGradRow floats apart -- an odd
// multiple of 16, so that the four partners of a quad fall in disjoint quarters of the 64 LDS
// banks while the 16 lanes of each read 16 consecutive words; the own copies of the column
// tiles are rows of NC + 1 floats (an odd stride, one bank per own point).
template <int KT, int DIM>
struct GradLds {
  static constexpr int NC = KT * DIM;
  static constexpr int kRow = ((2 * NC + 15) / 16) | 1;
  static constexpr int ROWF = 16 * kRow;          // floats per staged partner
  static constexpr int OWNF = NC + 1;             // floats per own point
};

template <int DIM, int KT, bool ROW>
__device__ void bgrad_tile(const ot_batch_desc& d, int first, int wv, int lane, double* wvals,
                           float* sh_pts, float* sh_pot, float* sh_own, double* sh_S) {
  using L = GradLds<KT, DIM>;
  constexpr int NC = L::NC;                   // output columns (block, component)
  constexpr int NCT = (NC + 15) / 16;         // column tiles of the matrix product
  constexpr int NS = NCT <= 2 ? 2 : 1;        // accumulator sets (alternating shifts)
  constexpr int RF = L::ROWF, OF = L::OWNF;
  static_assert((KT & (KT - 1)) == 0 && KT >= 1 && KT <= 32, "K a power of two up to 32");
  const int m = bm(d), K = d.K;
  const float s2 = (float)(kLog2eD / d.eps);
  const float eps = (float)d.eps;
  gcfloat* x = as_global(d.x);
  gcfloat* y = as_global(d.y);
  gcfloat* fpot = as_global(d.f);
  gcfloat* gpot = as_global(d.g);
  float* __restrict__ gout = ROW ? d.dx : d.dy;
  const bool grad = gout != nullptr;
  const int r16 = lane & 15, iq = lane >> 4;
  const int o0 = first + wv * kMfPts;          // the wave's first own point
  const bool actA = o0 + r16 < m;              // own point of this lane's A entries
  const int oc = actA ? o0 + r16 : 0;
  const float po = ROW ? fpot[oc] : gpot[oc];
  float xo[DIM];
  if constexpr (ROW) {
#pragma unroll
    for (int dd = 0; dd < DIM; ++dd) xo[dd] = x[oc * DIM + dd];
  } else {
    // the own columns' copies y_{k m + j} of every block
    float* own = sh_own + (size_t)wv * kMfPts * OF;
    for (int e = lane; e < kMfPts * NC; e += kWave) {
      const int q = e / NC, kd = e - q * NC;
      const int o = min(o0 + q, m - 1);
      own[q * OF + kd] = y[((kd / DIM) * m + o) * DIM + kd % DIM];
    }
  }
  // this lane's B column in each tile (block r, component d as r DIM + d); the padding columns
  // of a last partial tile read a valid column and their results are not stored
  int bcol[NCT];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) bcol[ct] = min(ct * 16 + r16, NC - 1) + (ROW ? 0 : NC);
  v4d acc[NS][NCT];
#pragma unroll
  for (int u = 0; u < NS; ++u)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) acc[u][ct] = v4d{0.0, 0.0, 0.0, 0.0};
  // value sums: float64 per plan entry for the marginal, float32 over the K shifts of a
  // partner for P and <C, T> (then float64), as the point-per-wave path accumulates them
  double S = 0.0, tP = 0.0, tC = 0.0;
  gcfloat* src = ROW ? y : x;
  const float* own = sh_own + ((size_t)wv * kMfPts + r16) * OF;
#pragma unroll 1
  for (int c0 = 0; c0 < m; c0 += kGradChunk) {
    __syncthreads();  // the previous chunk's readers are done
    const int nc = min(kGradChunk, m - c0);
    for (int e = threadIdx.x; e < NC * kGradChunk; e += blockDim.x) {
      const int q = e % kGradChunk, cd = e / kGradChunk;
      const int cb = cd / DIM, dd = cd - cb * DIM;
      const float v = q < nc ? src[(cb * m + c0 + q) * DIM + dd] : 0.0f;
      sh_pts[q * RF + cd] = v;
      sh_pts[q * RF + cd + NC] = v;
    }
    if (threadIdx.x < kGradChunk)
      sh_pot[threadIdx.x] = (int)threadIdx.x < nc ? (ROW ? gpot : fpot)[c0 + threadIdx.x] : 0.0f;
    __syncthreads();
#pragma unroll 1
    for (int jq = 0; jq < nc; jq += 4) {
      const int jl = jq + iq;  // this lane's partner (A inner index and B row), < kGradChunk
      const float fg = po + sh_pot[jl];
      // exponent (fg - c) s2 as one FMA; -inf (T = 0) for an own point or partner beyond m
      const float fgs = actA && jl < nc ? fg * s2 : -INFINITY;
      const float* pp = sh_pts + jl * RF;
      float vP = 0.0f, vC = 0.0f;
      // (unrolled by two: a full unroll holds 254 registers at K = 32, dim 3 for the same time)
#pragma unroll 2
      for (int k = 0; k < KT; ++k) {
        float c = 0.0f;
#pragma unroll
        for (int dd = 0; dd < DIM; ++dd) {
          const float e = ROW ? xo[dd] - pp[k * DIM + dd] : pp[dd] - own[k * DIM + dd];
          c = fmaf(e, e, c);
        }
        const float T = exp2_fast(fmaf(c, -s2, fgs));
        const double a = (double)T;
        S += a;
        if (ROW) {
          vP = fmaf(T, fg - eps, vP);  // T (C + eps (Z - 1)) = T (f + g - eps)
          vC = fmaf(T, c, vC);
        }
        // (run also when this pass has no gradient output: the products are then unused)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          // row: block (r + k) mod K at r DIM + d + k DIM; column: block (c - k) mod K at
          // c DIM + d + NC - k DIM (bcol holds the NC)
          const double b = (double)pp[bcol[ct] + (ROW ? k * DIM : -k * DIM)];
          acc[k % NS][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k % NS][ct], 0, 0, 0);
        }
      }
      if (ROW) {
        tP += (double)vP;
        tC += (double)vC;
      }
    }
  }
  // own point r16's sums: its four lanes (one per partner of a quad)
  S += __shfl_xor(S, 16, kWave);
  S += __shfl_xor(S, 32, kWave);
  tP += __shfl_xor(tP, 16, kWave);
  tP += __shfl_xor(tP, 32, kWave);
  tC += __shfl_xor(tC, 16, kWave);
  tC += __shfl_xor(tC, 32, kWave);
  if (iq == 0) sh_S[wv * kMfPts + r16] = S;
  __syncthreads();
  if (grad) {
    // lane l holds the sums of own points o0 + l / 16 + 4 v for its column of each tile
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      v4d D = acc[0][ct];
      if constexpr (NS == 2) D += acc[1][ct];
      const int col = ct * 16 + r16;
      if (col >= NC) continue;
      const int r = col / DIM, dd = col - r * DIM;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int q = iq + 4 * v;
        const int o = o0 + q;
        if (o >= m) continue;
        const int Pi = r * m + o;
        const double ownc = (double)(ROW ? x : y)[Pi * DIM + dd];
        gout[Pi * DIM + dd] = (float)(2.0 * (ownc * sh_S[wv * kMfPts + q] - D[v]));
      }
    }
  }
  // per own point: folded marginal, da / db, and the value terms (lanes 0..15)
  gcfloat* marg_in = as_global(ROW ? d.a : d.b);
  gcfloat* pot = ROW ? fpot : gpot;
  double ps = 0.0;
  for (int q = lane; q < m; q += kWave) ps += (double)pot[q];
  const double pmean = wave_sum_all_d(ps) / m;
  float* __restrict__ dpot = ROW ? d.da : d.db;
  double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0, v4 = 0.0;
  if (iq == 0 && actA) {
    const int o = o0 + r16;
    double mv = 0.0;
    for (int r = 0; r < K; ++r) mv += (double)marg_in[r * m + o];
    const double marg = mv / K;
    if (dpot)
      for (int r = 0; r < K; ++r) dpot[r * m + o] = (float)((double)po - pmean);
    const double dr = S - marg;
    v0 = ROW ? tP : 0.0;
    v1 = ROW ? tC : 0.0;
    v2 = ROW ? S : 0.0;
    v3 = dr * dr;
    v4 = (double)po * marg;
  }
  v0 = wave_sum_all_d(v0);
  v1 = wave_sum_all_d(v1);
  v2 = wave_sum_all_d(v2);
  v3 = wave_sum_all_d(v3);
  v4 = wave_sum_all_d(v4);
  if (lane == 0) {
    wvals[0] = v0;
    wvals[1] = v1;
    wvals[2] = v2;
    wvals[3] = v3;
    wvals[4] = v4;
  }
}

// Values only (a problem whose descriptor asks for no coordinate gradients): each wave takes
// four own points, so that a staged partner chunk serves the workgroup's sixteen points; per
// point the row (column) sum, P and <C, T> of the K m plan entries of block 0, da / db and
// the marginal terms, as badj_point.
constexpr int kValPts = 4;  // own points per wave in values-only tiles

template <int DIM, int KT>
__device__ void bval_points(const ot_batch_desc& d, int o0, int lane, int wv,
                            double (*vals)[8], float* sh_pts, float* sh_pot, double* sh_cols,
                            double* __restrict__ colpart) {
  const int m = bm(d), K = d.K;
  const float s2 = (float)(kLog2eD / d.eps);
  gcfloat* x = as_global(d.x);
  gcfloat* y = as_global(d.y);
  gcfloat* fpot = as_global(d.f);
  gcfloat* gpot = as_global(d.g);
  float po[kValPts], xo[kValPts][DIM];
  bool act[kValPts];
#pragma unroll
  for (int q = 0; q < kValPts; ++q) {
    act[q] = o0 + q < m;
    const int oc = act[q] ? o0 + q : 0;
    po[q] = fpot[oc];
#pragma unroll
    for (int dd = 0; dd < DIM; ++dd) xo[q][dd] = x[oc * DIM + dd];
  }
  double S[kValPts] = {};
  float vC[kValPts] = {};
#pragma unroll 1
  for (int c0 = 0; c0 < m; c0 += kAdjChunk) {
    __syncthreads();  // the previous chunk's readers are done
    const int nc = min(kAdjChunk, m - c0);
    // the partners' copies in every block (the costs' y_{k m + j})
    for (int e = threadIdx.x; e < KT * DIM * kAdjChunk; e += blockDim.x) {
      const int qq = e % kAdjChunk, cd = e / kAdjChunk;
      const int cb = cd / DIM, dd = cd - cb * DIM;
      sh_pts[e] = qq < nc ? y[(cb * m + c0 + qq) * DIM + dd] : 0.0f;
    }
    if (threadIdx.x < kAdjChunk)
      sh_pot[threadIdx.x] = (int)threadIdx.x < nc ? gpot[c0 + threadIdx.x] : 0.0f;
    __syncthreads();
    double col = 0.0;  // the lane's column j = c0 + lane: its terms over the wave's rows
    if (lane < nc) {
      const float pp = sh_pot[lane];
      float fgs[kValPts];  // exponent (f_i + g_j - c) s2 as one FMA per entry
#pragma unroll
      for (int q = 0; q < kValPts; ++q) fgs[q] = (po[q] + pp) * s2;
#pragma unroll 2
      for (int k = 0; k < KT; ++k) {
        float pt[DIM];
#pragma unroll
        for (int dd = 0; dd < DIM; ++dd) pt[dd] = sh_pts[(k * DIM + dd) * kAdjChunk + lane];
#pragma unroll
        for (int q = 0; q < kValPts; ++q) {
          float c = 0.0f;
#pragma unroll
          for (int dd = 0; dd < DIM; ++dd) {
            const float e = xo[q][dd] - pt[dd];
            c = fmaf(e, e, c);
          }
          const float T = act[q] ? exp2_fast(fmaf(c, -s2, fgs[q])) : 0.0f;
          const double Td = (double)T;
          S[q] += Td;
          col += Td;
          vC[q] = fmaf(T, c, vC[q]);
        }
      }
    }
    // the tile's partial column sums: the four waves' through LDS, one store per column
    sh_cols[wv * kWave + lane] = col;
    __syncthreads();
    if (wv == 0 && lane < nc) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kAdjPts; ++w) t += sh_cols[w * kWave + lane];
      colpart[c0 + lane] = t;
    }
  }
  gcfloat* marg_in = as_global(d.a);
  double ps = 0.0;
  for (int qq = lane; qq < m; qq += kWave) ps += (double)fpot[qq];
  const double pmean = wave_sum_all_d(ps) / m;
  float* __restrict__ dpot = d.da;
#pragma unroll
  for (int q = 0; q < kValPts; ++q) {
    const double Sq = wave_sum_all_d(S[q]);
    const double tC = wave_sum_all_d((double)vC[q]);
    if (!act[q]) continue;
    const int o = o0 + q;
    double mv = 0.0;
    for (int r = lane; r < K; r += kWave) mv += (double)marg_in[r * m + o];
    const double marg = wave_sum_all_d(mv) / K;
    if (dpot)
      for (int r = lane; r < K; r += kWave) dpot[r * m + o] = (float)((double)po[q] - pmean);
    if (lane == 0) {
      const double dr = Sq - marg;
      // sum_{j,k} T_ijk (f_i + g_j - eps) = (f_i - eps) rowsum_i + (the g_j colsum_j terms,
      // added by batched_finalize_kernel from the column sums)
      vals[q][0] = ((double)po[q] - d.eps) * Sq;
      vals[q][1] = tC;
      vals[q][2] = Sq;
      vals[q][3] = dr * dr;
      vals[q][4] = (double)po[q] * marg;
    }
  }
}

// Without coordinate gradients (and K with its own instantiation) a problem has only row
// tiles: the column sums are accumulated in the same pass, each tile's partial per column
// stored in the problem's folded-kernel scratch (no longer needed after the solve) as
// colpart[tile][m] doubles, and the column statistics finished by batched_finalize_kernel.
__host__ __device__ __forceinline__ bool fused_columns(const ot_batch_desc& d, bool kt) {
  return d.dx == nullptr && d.dy == nullptr && kt;
}
__device__ __forceinline__ double* colpart_base(const ot_batch_desc& d) {
  return reinterpret_cast<double*>(d.logK);
}

// Value tiles are grouped by (dim, K) class so that each class runs its own instantiation
// (its own register allocation): the launch for a class covers the tiles [tile0, tile0 +
// grid) of the problems vorder[0 .. nq), whose first tiles vstart[] increase.
//
// VO selects the values-only problems of the class (with their fused column sums); the other
// instantiation serves the problems with coordinate gradients.  Both are launched over the
// class's tiles and a tile of the other kind returns at once, so each has its own register
// allocation.
template <int DIM, int KT, bool VO>
__global__ void __launch_bounds__(256)
    batched_values_kernel(const ot_batch_desc* __restrict__ descs,
                          const int32_t* __restrict__ vorder, const int32_t* __restrict__ vstart,
                          int nq, int tile0, double* __restrict__ accs) {
  __shared__ double vals16[kAdjPts * kValPts][8];
  const int tile = tile0 + (int)blockIdx.x;
  const int q = find_problem(vstart, nq, tile);
  const int p = vorder[q];
  const ot_batch_desc d = descs[p];
  const int m = bm(d);
  // gradients: 4 own points per tile (one per wave); values only: 16 (four per wave)
  const bool grad = d.dx != nullptr || d.dy != nullptr;
  if ((!grad && KT > 0) != VO) return;
  const int ppt = VO ? kAdjPts * kValPts : (KT > 0 ? kGradPts : kAdjPts);
  const int nrow = (m + ppt - 1) / ppt;
  const int t = tile - vstart[q];
  double* acc = accs + 8 * (size_t)p;
  const bool row = t < nrow;  // values only: every tile is a row tile
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int first = (row ? t : t - nrow) * ppt;
  if constexpr (!VO && KT > 0) {
    // 16 own points per wave on the matrix cores; LDS sized for the class
    using L = GradLds<KT, DIM>;
    __shared__ float g_pts[kGradChunk * L::ROWF];
    __shared__ float g_pot[kGradChunk];
    __shared__ float g_own[kAdjPts * kMfPts * L::OWNF];  // column tiles' own copies
    __shared__ double g_S[kGradPts];
    if (lane == 0)
      for (int v = 0; v < 8; ++v) vals16[wv][v] = 0.0;
    if (row)
      bgrad_tile<DIM, KT, true>(d, first, wv, lane, vals16[wv], g_pts, g_pot, g_own, g_S);
    else
      bgrad_tile<DIM, KT, false>(d, first, wv, lane, vals16[wv], g_pts, g_pot, g_own, g_S);
  } else if constexpr (!VO) {
    // generic K: one own point per wave
    const int o = first + wv;
    const bool active = o < m;
    if (lane == 0)
      for (int v = 0; v < 8; ++v) vals16[wv][v] = 0.0;
    if (row) badj_point<DIM, true>(d, o, active, lane, vals16[wv]);
    else badj_point<DIM, false>(d, o, active, lane, vals16[wv]);
  } else {
    // row tiles only (the column sums in the same pass); LDS sized for the class
    __shared__ float vo_pts[(KT > 0 ? KT : 1) * DIM * kAdjChunk];
    __shared__ float vo_pot[kAdjChunk];
    __shared__ double vo_cols[kAdjPts * kWave];
    const int o0 = first + wv * kValPts;
    if (lane < kValPts)
      for (int v = 0; v < 8; ++v) vals16[wv * kValPts + lane][v] = 0.0;
    __syncthreads();
    bval_points<DIM, KT>(d, o0, lane, wv, &vals16[wv * kValPts], vo_pts, vo_pot, vo_cols,
                         colpart_base(d) + (size_t)t * m);
  }
  __syncthreads();
  // the workgroup's partials: one atomic add per value
  if (threadIdx.x < 5) {
    const int v = threadIdx.x;
    const int np = VO ? ppt : kAdjPts;  // one partial per wave with gradients
    double sum = 0.0;
    for (int w = 0; w < np; ++w) sum += vals16[w][v];
    // rows: P, <C,T>, mass, (rowsum - alpha)^2, <f,alpha>; columns: (colsum - beta)^2, <g,beta>
    const int slot = row ? (v < 4 ? v : 5) : (v == 3 ? 4 : v == 4 ? 6 : -1);
    if (slot >= 0) atomicAdd(&acc[slot], sum);
  }
}

// One workgroup per problem.  With the column sums fused into the row tiles it first
// finishes the column statistics from the tiles' partials: sum_j (colsum_j - beta_j)^2 and
// <g, beta>, beta the folded column marginal (float64 mean over the blocks).
__global__ void __launch_bounds__(1024)
    batched_finalize_kernel(const ot_batch_desc* __restrict__ descs,
                            const double* __restrict__ accs) {
  __shared__ double red[1024 / kWave];
  const int p = blockIdx.x;
  const ot_batch_desc d = descs[p];
  const double* acc = accs + 8 * (size_t)p;
  const int m = bm(d), Ki = d.K;
  const bool kt = Ki == 1 || Ki == 2 || Ki == 4 || Ki == 8 || Ki == 16 || Ki == 32;
  double col_err = acc[4], col_dual = acc[6], primal_cols = 0.0;
  if (fused_columns(d, kt)) {
    const int ntile = (m + kAdjPts * kValPts - 1) / (kAdjPts * kValPts);
    const double* colpart = colpart_base(d);
    double e2 = 0.0, gb = 0.0, gs = 0.0, gc = 0.0;
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
      double cp[4] = {0.0, 0.0, 0.0, 0.0};  // four partial sums: the loads overlap
      int t = 0;
      for (; t + 4 <= ntile; t += 4)
#pragma unroll
        for (int u = 0; u < 4; ++u) cp[u] += colpart[(size_t)(t + u) * m + j];
      for (; t < ntile; ++t) cp[0] += colpart[(size_t)t * m + j];
      const double cs = (cp[0] + cp[1]) + (cp[2] + cp[3]);
      double bm_ = 0.0;
      for (int r = 0; r < Ki; ++r) bm_ += (double)d.b[(int64_t)r * m + j];
      bm_ /= Ki;
      e2 += (cs - bm_) * (cs - bm_);
      gb += (double)d.g[j] * bm_;
      gs += (double)d.g[j];
      gc += (double)d.g[j] * cs;
    }
    col_err = block_sum_d(e2, red);
    col_dual = block_sum_d(gb, red);
    primal_cols = block_sum_d(gc, red);
    if (d.db) {  // dP/db = g - mean(g), tiled (written by the column tiles otherwise)
      const double gmean = block_sum_d(gs, red) / m;
      for (int e = threadIdx.x; e < Ki * m; e += blockDim.x)
        d.db[e] = (float)((double)d.g[e % m] - gmean);
    }
  }
  if (threadIdx.x == 0) {
    const double K = d.K;
    d.out[0] = K * (acc[0] + primal_cols);
    d.out[1] = K * (acc[5] + col_dual) - d.eps * K * acc[2];
    d.out[2] = K * acc[1];
    d.out[3] = sqrt(K * acc[3]);
    d.out[4] = sqrt(K * col_err);
  }
}

__global__ void zero_d_words(double* p, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// ---- host ----------------------------------------------------------------------------------
static size_t a256(size_t v) { return (v + 255) / 256 * 256; }

// Value-tile classes: (dim, K) with K in {1, 2, 4, 8, 16, 32} or any other K.
constexpr int kKClasses = 7;
constexpr int kVClasses = 2 * kKClasses;
static int k_class(int K) {
  switch (K) {
    case 1: return 0;
    case 2: return 1;
    case 4: return 2;
    case 8: return 3;
    case 16: return 4;
    case 32: return 5;
    default: return 6;
  }
}
static int v_class(int dim, int K) { return (dim == 3 ? kKClasses : 0) + k_class(K); }

// plan = {nfold, nval, count, ntasks, cls_q[kVClasses + 1], cls_tile[kVClasses + 1],
//         cls_kind[kVClasses], order[count], fold_start[count], vorder[count], vstart[count],
//         tasks[ntasks]}:
// cls_kind[c] bit 0: the class has problems with coordinate gradients, bit 1: values-only ones;
// fold_start[q] is the first fold tile of problem order[q];
// problems of value class c are vorder[cls_q[c] .. cls_q[c + 1]), their value tiles
// [cls_tile[c], cls_tile[c + 1]); vstart[q] is the first value tile of vorder[q].
constexpr int kPlanHead = 4 + 2 * (kVClasses + 1) + kVClasses;

size_t batched_plan_len(int count) {
  return kPlanHead + (4 + (size_t)kMaxGangF) * (size_t)count;
}

// Workgroups that solve one problem together: one up to m = 256 (logK then costs a single
// workgroup at most ~0.1 ms per solve), about 128 rows per member above.
static int gang_size(int m) {
  if (m <= 256) return 1;
  const int g = (m + 127) / 128;
  return g < kMaxGangF ? g : kMaxGangF;
}

// tasks: problem | member << 20 | (G - 1) << 26, largest problems first, the G members of a
// gang consecutive.
int batched_plan(const ot_batch_desc* h, int count, int32_t* plan) {
  if (count >= (1 << 20)) return -1;
  std::vector<int> idx(count);
  for (int p = 0; p < count; ++p) idx[p] = p;
  auto cost = [&](int p) {
    const double m = (double)h[p].n / h[p].K;
    return m * m * (1.0 + 0.05 * h[p].K);  // iterations ~ m^2 each; fold ~ K m^2 once
  };
  std::stable_sort(idx.begin(), idx.end(), [&](int u, int v) { return cost(u) > cost(v); });
  int32_t* cls_q = plan + 4;
  int32_t* cls_tile = cls_q + kVClasses + 1;
  int32_t* cls_kind = cls_tile + kVClasses + 1;
  int32_t* order = plan + kPlanHead;
  int32_t* fstart = order + count;
  int32_t* vorder = fstart + count;
  int32_t* vstart = vorder + count;
  uint32_t* tasks = reinterpret_cast<uint32_t*>(vstart + count);
  int64_t nf = 0, nv = 0;
  int nt = 0;
  for (int q = 0; q < count; ++q) {  // fold tiles in the solve order: the largest first
    order[q] = idx[q];
    const int m = h[idx[q]].n / h[idx[q]].K;
    fstart[q] = (int32_t)nf;
    nf += (int64_t)fold_row_blocks(m) * fold_col_blocks(m, h[idx[q]].tile_cfg);
  }
  // value tiles by class, the largest problems first within a class (their tiles run longest,
  // so that the small ones fill the end of the launch), then in index order
  std::vector<int> vo(count);
  for (int p = 0; p < count; ++p) vo[p] = p;
  std::stable_sort(vo.begin(), vo.end(), [&](int u, int v) {
    const int cu = v_class(h[u].dim, h[u].K), cv = v_class(h[v].dim, h[v].K);
    if (cu != cv) return cu < cv;
    return h[u].n / h[u].K > h[v].n / h[v].K;
  });
  int q = 0;
  for (int c = 0; c < kVClasses; ++c) {
    cls_q[c] = q;
    cls_tile[c] = (int32_t)nv;
    cls_kind[c] = 0;
    while (q < count && v_class(h[vo[q]].dim, h[vo[q]].K) == c) {
      const int p = vo[q];
      const int m = h[p].n / h[p].K;
      vorder[q] = p;
      vstart[q] = (int32_t)nv;
      // value tiles of block-0 points: with gradients 64 (16 per wave, matrix cores), or 4
      // (one per wave) when K takes the generic path; 16 without (four per wave)
      const bool kt = k_class(h[p].K) < 6;
      const int ppt = fused_columns(h[p], kt) ? kAdjPts * kValPts : (kt ? kGradPts : kAdjPts);
      nv += (fused_columns(h[p], kt) ? 1 : 2) * ((m + ppt - 1) / ppt);
      cls_kind[c] |= fused_columns(h[p], kt) ? 2 : 1;
      ++q;
    }
  }
  cls_q[kVClasses] = q;
  cls_tile[kVClasses] = (int32_t)nv;
  for (int r = 0; r < count; ++r) {
    const int p = idx[r];
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

template <int DIM, int KT>
static void launch_values_class(const ot_batch_desc* descs, const int32_t* vorder,
                                const int32_t* vstart, int q0, int q1, int t0, int t1,
                                int kind, double* accs, hipStream_t s) {
  if (kind & 1)
    hipLaunchKernelGGL((batched_values_kernel<DIM, KT, false>), dim3(t1 - t0), dim3(256), 0, s,
                       descs, vorder + q0, vstart + q0, q1 - q0, t0, accs);
  if constexpr (KT > 0)
    if (kind & 2)
      hipLaunchKernelGGL((batched_values_kernel<DIM, KT, true>), dim3(t1 - t0), dim3(256), 0, s,
                         descs, vorder + q0, vstart + q0, q1 - q0, t0, accs);
}

hipError_t launch_batched(const ot_batch_desc* descs, int count, const int32_t* dplan,
                          const int32_t* hplan, double tol, int max_iter, int fold_fp64,
                          int warm, void* ws, hipStream_t s, hipEvent_t* events) {
  char* base = static_cast<char*>(ws);
  uint32_t* queue = reinterpret_cast<uint32_t*>(base);
  double* accs = reinterpret_cast<double*>(base + a256(256));
  hipError_t e = launch_zero_words(queue, 64, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(zero_d_words, dim3(64), dim3(256), 0, s, accs, (int64_t)8 * count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int nfold = hplan[0];
  const int32_t* cls_q = hplan + 4;
  const int32_t* cls_tile = cls_q + kVClasses + 1;
  const int32_t* cls_kind = cls_tile + kVClasses + 1;
  const int32_t* order = dplan + kPlanHead;
  const int32_t* fstart = order + count;
  const int32_t* vorder = fstart + count;
  const int32_t* vstart = vorder + count;
  if (fold_fp64 != 0)
    hipLaunchKernelGGL(batched_fold_kernel<true>, dim3(nfold), dim3(kFoldThreads), 0, s, descs,
                       count, order, fstart);
  else
    hipLaunchKernelGGL(batched_fold_kernel<false>, dim3(nfold), dim3(kFoldThreads), 0, s, descs,
                       count, order, fstart);
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
  // the device copy of the plan: task count in entry 3, tasks after vstart
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
  // values and gradients: one launch per non-empty (dim, K) class
  for (int c = 0; c < kVClasses; ++c) {
    const int q0 = cls_q[c], q1 = cls_q[c + 1], t0 = cls_tile[c], t1 = cls_tile[c + 1];
    if (t1 <= t0) continue;
#define CSOT_VCLS(D, KT) \
  launch_values_class<D, KT>(descs, vorder, vstart, q0, q1, t0, t1, cls_kind[c], accs, s)
    switch (c) {
      case 0: CSOT_VCLS(2, 1); break;
      case 1: CSOT_VCLS(2, 2); break;
      case 2: CSOT_VCLS(2, 4); break;
      case 3: CSOT_VCLS(2, 8); break;
      case 4: CSOT_VCLS(2, 16); break;
      case 5: CSOT_VCLS(2, 32); break;
      case 6: CSOT_VCLS(2, 0); break;
      case 7: CSOT_VCLS(3, 1); break;
      case 8: CSOT_VCLS(3, 2); break;
      case 9: CSOT_VCLS(3, 4); break;
      case 10: CSOT_VCLS(3, 8); break;
      case 11: CSOT_VCLS(3, 16); break;
      case 12: CSOT_VCLS(3, 32); break;
      default: CSOT_VCLS(3, 0); break;
    }
#undef CSOT_VCLS
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(batched_finalize_kernel, dim3(count), dim3(1024), 0, s, descs, accs);
  return hipGetLastError();
}

}  // namespace csot
