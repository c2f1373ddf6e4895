// Fold of the Gibbs kernel over the K cyclic shifts, fold of the marginals, and the
// block-circulant projection of a cost.
//
//   logK_ij = log sum_k exp(-C_ijk / eps)           (eq. def_Kij; Alg. 2, first step)
//   alpha_i = (1/K) sum_r a_{r m + i}                (Alg. 3, stage 1)
//   Csym[i, k m + j] = (1/K) sum_r C[r m + i, ((r + k) mod K) m + j]
//
// C_ijk is block-row 0 of the block-circulant cost (eq. blkstr_cost): the cost between point
// i and point k*m + j, recomputed from the float32 coordinates or read from a dense C.  The
// k-sum is a max-shifted log-sum-exp: two passes over k (minimum cost, then the shifted sum),
// so no term overflows and the dominant term is exact.  In float64 mode the costs and the
// shifted exponents are float64 and only the exponentials of the (non-positive) shifted
// exponents run in float32, which keeps the result accurate to float32 rounding; in float32
// mode everything is float32, and the rounding of C / eps grows with its magnitude.
//
// Work per output entry: K cost evaluations twice and K exponentials; the output is m*m
// floats, so the kernel is bound by exp throughput (float32) or float64 FMA throughput.
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace csot {

__global__ void zero_words_kernel(uint32_t* p, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
    p[i] = 0u;
}

hipError_t launch_zero_words(uint32_t* p, int count, hipStream_t s) {
  const int blocks = (count + 255) / 256 < 64 ? (count + 255) / 256 : 64;
  hipLaunchKernelGGL(zero_words_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, p,
                     count);
  return hipGetLastError();
}

constexpr int kFoldTJ = 64;  // j per block (one wave wide -> coalesced reads of y / C)
constexpr int kFoldTI = 4;   // i per block

template <int DIM, typename Real>
__device__ __forceinline__ Real pt_cost(const float* __restrict__ x, int I,
                                        const float* __restrict__ y, int J) {
  Real c = 0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const Real df = (Real)x[(int64_t)I * DIM + d] - (Real)y[(int64_t)J * DIM + d];
    c += df * df;
  }
  return c;
}

// float64 costs, minimum and shifted exponents; the exponentials of the shifted exponents
// (all <= 0, the largest exactly 0) in float32 on the transcendental unit, the sum of at most
// K terms in [0, 1] in float32 (it lies in [1, K]) and the final sum in float64.  The result
// is accurate to float32 rounding of logK: the shift removes the large magnitude exactly.
template <int DIM>
__device__ __forceinline__ void fold_entry_fp64(const Geom& g, int i, int j, float* out) {
  double cmin = 1.0e300;
  for (int k = 0; k < g.K; ++k) {
    double c;
    if constexpr (DIM == 0) c = (double)g.C[(int64_t)i * g.ldc + (int64_t)k * g.m + j];
    else c = pt_cost<DIM, double>(g.x, i, g.y, k * g.m + j);
    cmin = c < cmin ? c : cmin;
  }
  const double s2 = kLog2eD / g.eps;
  float s = 0.0f;
  for (int k = 0; k < g.K; ++k) {
    double c;
    if constexpr (DIM == 0) c = (double)g.C[(int64_t)i * g.ldc + (int64_t)k * g.m + j];
    else c = pt_cost<DIM, double>(g.x, i, g.y, k * g.m + j);
    s += exp2_fast((float)((cmin - c) * s2));
  }
  *out = (float)(-cmin / g.eps + (double)log2_fast(s) * kLn2D);
}

template <int DIM>
__device__ __forceinline__ void fold_entry_fp32(const Geom& g, int i, int j, float s2,
                                                float* out) {
  float cmin = 3.0e38f;
  for (int k = 0; k < g.K; ++k) {
    float c;
    if constexpr (DIM == 0) c = g.C[(int64_t)i * g.ldc + (int64_t)k * g.m + j];
    else c = pt_cost<DIM, float>(g.x, i, g.y, k * g.m + j);
    cmin = fminf(c, cmin);
  }
  float s = 0.0f;
  for (int k = 0; k < g.K; ++k) {
    float c;
    if constexpr (DIM == 0) c = g.C[(int64_t)i * g.ldc + (int64_t)k * g.m + j];
    else c = pt_cost<DIM, float>(g.x, i, g.y, k * g.m + j);
    s += exp2_fast((cmin - c) * s2);
  }
  *out = (-cmin * s2 + log2_fast(s)) * kLn2;
}

constexpr int kFoldKC = 32;  // shifts k whose target points are staged in LDS at a time

// Blocks with blockIdx.y < ceil(m / TI) fold logK; the last row of blocks folds a and b.
// Point clouds: the block's 64 target columns j of up to 32 shifts k (points k m + j) are
// staged in LDS and every thread keeps its x_i in registers, so each cost is two LDS reads and
// a few FMAs; with K <= 32 one staging serves both passes over k.  Dense costs are read
// straight from C (no reuse across the block).
template <int DIM, bool FP64>
__global__ void __launch_bounds__(kFoldTJ* kFoldTI)
    fold_kernel(Geom g, float* __restrict__ logK, float* __restrict__ alpha,
                float* __restrict__ beta, int iblocks) {
  const int tj = threadIdx.x % kFoldTJ;
  const int ti = threadIdx.x / kFoldTJ;
  if ((int)blockIdx.y == iblocks) {
    // marginal fold: 2*m outputs over the x-dimension of this block row
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 2 * g.m) {
      const float* v = t < g.m ? g.a : g.b;
      const int i = t < g.m ? t : t - g.m;
      double acc = 0.0;
      for (int r = 0; r < g.K; ++r) acc += (double)v[(int64_t)r * g.m + i];
      (t < g.m ? alpha : beta)[i] = (float)(acc / (double)g.K);
    }
    return;
  }
  const int j0 = blockIdx.x * kFoldTJ;
  const int j = j0 + tj;
  const int i = blockIdx.y * kFoldTI + ti;
  if constexpr (DIM == 0) {
    if (i >= g.m || j >= g.m) return;
    float* out = logK + (int64_t)i * g.m + j;
    if constexpr (FP64) fold_entry_fp64<DIM>(g, i, j, out);
    else fold_entry_fp32<DIM>(g, i, j, (float)(kLog2eD / g.eps), out);
  } else {
    using Real = typename std::conditional<FP64, double, float>::type;
    __shared__ float ys[kFoldKC][DIM][kFoldTJ];
    const bool active = i < g.m && j < g.m;  // inactive threads still stage and meet barriers
    Real xi[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) xi[d] = active ? (Real)g.x[(int64_t)i * DIM + d] : Real(0);
    const int nkc = (g.K + kFoldKC - 1) / kFoldKC;
    auto stage = [&](int kc) {
      const int kb = kc * kFoldKC;
      const int nk = min(kFoldKC, g.K - kb);
      for (int e = threadIdx.x; e < nk * kFoldTJ; e += blockDim.x) {
        const int kk = e / kFoldTJ, t = e - kk * kFoldTJ;
        const int jj = j0 + t;
#pragma unroll
        for (int d = 0; d < DIM; ++d)
          ys[kk][d][t] = jj < g.m ? g.y[((int64_t)(kb + kk) * g.m + jj) * DIM + d] : 0.0f;
      }
    };
    // C_ijk = |x_i - y_{k m + j}|^2 (exact in float64 for float32 inputs)
    auto cost = [&](int kk) {
      Real c = 0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const Real df = xi[d] - (Real)ys[kk][d][tj];
        c += df * df;
      }
      return c;
    };
    // pass 1: the minimum cost over k; pass 2: the shifted sum (one staging when K <= 32)
    Real cmin = FP64 ? Real(1.0e300) : Real(3.0e38f);
    for (int kc = 0; kc < nkc; ++kc) {
      if (kc > 0) __syncthreads();  // the previous chunk's readers are done
      stage(kc);
      __syncthreads();
      const int nk = min(kFoldKC, g.K - kc * kFoldKC);
      if (active)
        for (int kk = 0; kk < nk; ++kk) {
          const Real c = cost(kk);
          cmin = c < cmin ? c : cmin;
        }
    }
    const Real s2 = (Real)(kLog2eD / g.eps);
    float sum = 0.0f;
    for (int kc = 0; kc < nkc; ++kc) {
      if (nkc > 1) {
        __syncthreads();
        stage(kc);
        __syncthreads();
      }
      const int nk = min(kFoldKC, g.K - kc * kFoldKC);
      if (active)
        for (int kk = 0; kk < nk; ++kk) sum += exp2_fast((float)((cmin - cost(kk)) * s2));
    }
    if (active) {
      float* out = logK + (int64_t)i * g.m + j;
      if constexpr (FP64) *out = (float)(-cmin / g.eps + (double)log2_fast(sum) * kLn2D);
      else *out = (-cmin * s2 + log2_fast(sum)) * kLn2;
    }
  }
}

// Point clouds with float64 costs: the square expanded, -C_ijk s2 = -s2 |x_i|^2 + u_k with
// u_k = a_i . y_{k m + j} - P_kj, a_i = 2 s2 x_i, P_kj = s2 |y_{k m + j}|^2, all in float64
// (the expansion loses nothing visible at float32 output: its rounding is ~1e-16 of
// s2 |x| |y|).  The block's 64 columns j of up to 32 shifts are staged in LDS as float64 with
// their P, and each thread folds kFoldRPT rows of its column, so a staged value serves them
// all: a term costs DIM FMAs and a max in the first pass and DIM FMAs, an add, the conversion
// and the exponential in the second.  logK_ij = ln 2 (-s2 |x_i|^2 + U + log2 sum_k 2^(u_k - U)),
// U = max_k u_k.
constexpr int kFoldRPT = 2;  // rows per thread

template <int DIM>
__global__ void __launch_bounds__(kFoldTJ* kFoldTI)
    fold_points_kernel(Geom g, float* __restrict__ logK, float* __restrict__ alpha,
                       float* __restrict__ beta, int iblocks) {
  const int tj = threadIdx.x % kFoldTJ;
  const int ti = threadIdx.x / kFoldTJ;
  if ((int)blockIdx.y == iblocks) {
    // marginal fold: 2*m outputs over the x-dimension of this block row
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 2 * g.m) {
      const float* v = t < g.m ? g.a : g.b;
      const int i = t < g.m ? t : t - g.m;
      double acc = 0.0;
      for (int r = 0; r < g.K; ++r) acc += (double)v[(int64_t)r * g.m + i];
      (t < g.m ? alpha : beta)[i] = (float)(acc / (double)g.K);
    }
    return;
  }
  __shared__ double ys[kFoldKC][DIM][kFoldTJ];
  __shared__ double ps[kFoldKC][kFoldTJ];
  const int m = g.m;
  const int j0 = blockIdx.x * kFoldTJ;
  const int j = j0 + tj;
  const int ib = blockIdx.y * (kFoldTI * kFoldRPT) + ti * kFoldRPT;
  const double s2 = kLog2eD / g.eps;
  double a[kFoldRPT][DIM], xx[kFoldRPT], U[kFoldRPT];
  float sum[kFoldRPT];
#pragma unroll
  for (int q = 0; q < kFoldRPT; ++q) {
    const int ic = min(ib + q, m - 1);
    double n2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double xv = (double)g.x[(int64_t)ic * DIM + d];
      a[q][d] = 2.0 * s2 * xv;
      n2 = fma(xv, xv, n2);
    }
    xx[q] = s2 * n2;
    U[q] = -1.0e300;
    sum[q] = 0.0f;
  }
  const int nkc = (g.K + kFoldKC - 1) / kFoldKC;
  auto stage = [&](int kc) {
    const int kb = kc * kFoldKC;
    const int nk = min(kFoldKC, g.K - kb);
    for (int e = threadIdx.x; e < nk * kFoldTJ; e += blockDim.x) {
      const int kk = e / kFoldTJ, t = e - kk * kFoldTJ;
      const int jj = j0 + t;
      double n2 = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double v = jj < m ? (double)g.y[((int64_t)(kb + kk) * m + jj) * DIM + d] : 0.0;
        ys[kk][d][t] = v;
        n2 = fma(v, v, n2);
      }
      ps[kk][t] = s2 * n2;
    }
  };
  // pass 1: U = max_k u_k
  for (int kc = 0; kc < nkc; ++kc) {
    if (kc > 0) __syncthreads();  // the previous chunk's readers are done
    stage(kc);
    __syncthreads();
    const int nk = min(kFoldKC, g.K - kc * kFoldKC);
    for (int kk = 0; kk < nk; ++kk) {
      double yv[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) yv[d] = ys[kk][d][tj];
      const double P = ps[kk][tj];
#pragma unroll
      for (int q = 0; q < kFoldRPT; ++q) {
        double u = -P;
#pragma unroll
        for (int d = 0; d < DIM; ++d) u = fma(a[q][d], yv[d], u);
        U[q] = u > U[q] ? u : U[q];
      }
    }
  }
  // pass 2: sum_k 2^(u_k - U) (one staging when K <= 32)
  for (int kc = 0; kc < nkc; ++kc) {
    if (nkc > 1) {
      __syncthreads();
      stage(kc);
      __syncthreads();
    }
    const int nk = min(kFoldKC, g.K - kc * kFoldKC);
    for (int kk = 0; kk < nk; ++kk) {
      double yv[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) yv[d] = ys[kk][d][tj];
      const double P = ps[kk][tj];
#pragma unroll
      for (int q = 0; q < kFoldRPT; ++q) {
        double t = -(P + U[q]);
#pragma unroll
        for (int d = 0; d < DIM; ++d) t = fma(a[q][d], yv[d], t);
        sum[q] += exp2_fast((float)t);
      }
    }
  }
  if (j < m) {
#pragma unroll
    for (int q = 0; q < kFoldRPT; ++q)
      if (ib + q < m)
        logK[(int64_t)(ib + q) * m + j] =
            (float)((U[q] - xx[q] + (double)log2_fast(sum[q])) * kLn2D);
  }
}

template <int DIM, bool FP64>
static hipError_t launch_fold_t(const Geom& g, float* logK, float* alpha, float* beta,
                                hipStream_t s) {
  const int jblocks = (g.m + kFoldTJ - 1) / kFoldTJ;
  const int mblocks = (2 * g.m + kFoldTJ * kFoldTI - 1) / (kFoldTJ * kFoldTI);
  const int gx = jblocks > mblocks ? jblocks : mblocks;
  if constexpr (DIM > 0 && FP64) {
    const int iblocks = (g.m + kFoldTI * kFoldRPT - 1) / (kFoldTI * kFoldRPT);
    hipLaunchKernelGGL((fold_points_kernel<DIM>), dim3(gx, iblocks + 1),
                       dim3(kFoldTJ * kFoldTI), 0, s, g, logK, alpha, beta, iblocks);
  } else {
    const int iblocks = (g.m + kFoldTI - 1) / kFoldTI;
    hipLaunchKernelGGL((fold_kernel<DIM, FP64>), dim3(gx, iblocks + 1), dim3(kFoldTJ * kFoldTI),
                       0, s, g, logK, alpha, beta, iblocks);
  }
  return hipGetLastError();
}

hipError_t launch_fold(const Geom& g, bool fp64, float* logK, float* alpha, float* beta,
                       hipStream_t s) {
  switch (g.dim) {
    case 0: return fp64 ? launch_fold_t<0, true>(g, logK, alpha, beta, s)
                        : launch_fold_t<0, false>(g, logK, alpha, beta, s);
    case 2: return fp64 ? launch_fold_t<2, true>(g, logK, alpha, beta, s)
                        : launch_fold_t<2, false>(g, logK, alpha, beta, s);
    case 3: return fp64 ? launch_fold_t<3, true>(g, logK, alpha, beta, s)
                        : launch_fold_t<3, false>(g, logK, alpha, beta, s);
    default: return hipErrorInvalidValue;
  }
}

// ---- block-circulant projection ----------------------------------------------------------
// One thread per output entry (i, j) of block k = blockIdx.z; float64 accumulation of the K
// float32 costs along the block diagonal.
template <int DIM>
__global__ void __launch_bounds__(kFoldTJ* kFoldTI)
    symmetrize_kernel(Geom g, float* __restrict__ Csym, int64_t ldcs) {
  const int j = blockIdx.x * kFoldTJ + threadIdx.x % kFoldTJ;
  const int i = blockIdx.y * kFoldTI + threadIdx.x / kFoldTJ;
  const int k = blockIdx.z;
  if (i >= g.m || j >= g.m) return;
  double acc = 0.0;
  for (int r = 0; r < g.K; ++r) {
    const int I = r * g.m + i;
    const int J = ((r + k) % g.K) * g.m + j;
    if constexpr (DIM == 0) acc += (double)g.C[(int64_t)I * g.ldc + J];
    else acc += (double)pt_cost<DIM, float>(g.x, I, g.y, J);
  }
  Csym[(int64_t)i * ldcs + (int64_t)k * g.m + j] = (float)(acc / (double)g.K);
}

hipError_t launch_symmetrize(const Geom& g, float* Csym, int64_t ldcs, hipStream_t s) {
  const dim3 grid((g.m + kFoldTJ - 1) / kFoldTJ, (g.m + kFoldTI - 1) / kFoldTI, g.K);
  const dim3 block(kFoldTJ * kFoldTI);
  switch (g.dim) {
    case 0: hipLaunchKernelGGL(symmetrize_kernel<0>, grid, block, 0, s, g, Csym, ldcs); break;
    case 2: hipLaunchKernelGGL(symmetrize_kernel<2>, grid, block, 0, s, g, Csym, ldcs); break;
    case 3: hipLaunchKernelGGL(symmetrize_kernel<3>, grid, block, 0, s, g, Csym, ldcs); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace csot
