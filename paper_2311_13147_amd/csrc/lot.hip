// Cyclic linear OT (Thm. 1, Alg. 1): the data-parallel steps around the small LP.
//
//   G_ij    = min_k C_ijk                       (eq. definition_G; Alg. 1, first step)
//   kmin_ij = the smallest k attaining it       (the tie rule stated with Thm. 1)
//   alpha_i = (1/K) sum_r a_{r m + i}, beta likewise (the small problem's marginals)
//
// and, once the caller has solved the small LP  min <G, S>  s.t.  S 1 = alpha, S^T 1 = beta,
//
//   T[r m + i, c m + j] = S_ij if (c - r) mod K == kmin_ij, else 0
//
// (eq. optimal_solution_problem_CLOT placed by Lemma 1; Alg. 1, last steps).  The full plan
// has the value K <G, S>, the full problem's optimum.
//
// The minimum decides an integer, so costs from coordinates are float64 with every product
// and sum rounded on its own (no fused multiply-add): the same arithmetic as a plain float64
// evaluation of sum_d (x_d - y_d)^2, which therefore picks the same k.  Dense costs are
// compared as given.  G is stored in float32.
#include "common.hpp"
#include "launch.hpp"

namespace csot {

constexpr int kLotTJ = 64;  // j per block (one wave wide)
constexpr int kLotTI = 4;   // i per block

template <int DIM>
__global__ void __launch_bounds__(kLotTJ* kLotTI)
    lot_fold_kernel(Geom g, float* __restrict__ G, int32_t* __restrict__ kmin,
                    float* __restrict__ alpha, float* __restrict__ beta, int iblocks) {
  if ((int)blockIdx.y == iblocks) {
    // marginal fold: 2 m outputs
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
  const int j = blockIdx.x * kLotTJ + threadIdx.x % kLotTJ;
  const int i = blockIdx.y * kLotTI + threadIdx.x / kLotTJ;
  if (i >= g.m || j >= g.m) return;
  double best = 0.0;
  int kb = 0;
  for (int k = 0; k < g.K; ++k) {
    double c;
    if constexpr (DIM == 0) {
      c = (double)g.C[(int64_t)i * g.ldc + (int64_t)k * g.m + j];
    } else {
      c = 0.0;
      const int64_t J = (int64_t)k * g.m + j;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const double df = (double)g.x[(int64_t)i * DIM + d] - (double)g.y[J * DIM + d];
        c = __dadd_rn(c, __dmul_rn(df, df));
      }
    }
    if (k == 0 || c < best) {  // strict: the first (smallest) k among equal minima
      best = c;
      kb = k;
    }
  }
  G[(int64_t)i * g.m + j] = (float)best;
  kmin[(int64_t)i * g.m + j] = kb;
}

hipError_t launch_lot_fold(const Geom& g, float* G, int32_t* kmin, float* alpha, float* beta,
                           hipStream_t s) {
  const int jblocks = (g.m + kLotTJ - 1) / kLotTJ;
  const int iblocks = (g.m + kLotTI - 1) / kLotTI;
  const int mblocks = (2 * g.m + kLotTJ * kLotTI - 1) / (kLotTJ * kLotTI);
  const dim3 grid(jblocks > mblocks ? jblocks : mblocks, iblocks + 1);
  const dim3 block(kLotTJ * kLotTI);
  switch (g.dim) {
    case 0: hipLaunchKernelGGL(lot_fold_kernel<0>, grid, block, 0, s, g, G, kmin, alpha, beta, iblocks); break;
    case 2: hipLaunchKernelGGL(lot_fold_kernel<2>, grid, block, 0, s, g, G, kmin, alpha, beta, iblocks); break;
    case 3: hipLaunchKernelGGL(lot_fold_kernel<3>, grid, block, 0, s, g, G, kmin, alpha, beta, iblocks); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Scatter of the small LP's solution: block (i, j, k) of the grid reads S_ij and kmin_ij once
// and writes the K entries T[r m + i, ((r + k) mod K) m + j], r = 0..K-1 (one per block row),
// four consecutive j per lane with non-temporal stores, like the entropic expansion.
constexpr int kLotExpTJ = 256;  // j per block row segment (64 lanes x 4)
constexpr int kLotExpTI = 4;    // i per block (one wave each)

template <bool VEC>
__global__ void __launch_bounds__(256)
    lot_expand_kernel(int m, int K, const float* __restrict__ S,
                      const int32_t* __restrict__ kmin, float* __restrict__ T, int64_t ldt) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.y * kLotExpTI + wv;
  const int k = blockIdx.z;
  const int j0 = blockIdx.x * kLotExpTJ + lane * 4;
  if (i >= m || j0 >= m) return;
  float v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = j0 + q;
    v[q] = (j < m && kmin[(int64_t)i * m + j] == k) ? S[(int64_t)i * m + j] : 0.0f;
  }
  for (int r = 0; r < K; ++r) {
    const int c = r + k < K ? r + k : r + k - K;
    float* dst = T + (int64_t)(r * m + i) * ldt + (int64_t)c * m + j0;
    if constexpr (VEC) {
      typedef float v4f __attribute__((ext_vector_type(4)));
      const v4f val = {v[0], v[1], v[2], v[3]};
      __builtin_nontemporal_store(val, reinterpret_cast<v4f*>(dst));
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (j0 + q < m) __builtin_nontemporal_store(v[q], dst + q);
    }
  }
}

hipError_t launch_lot_expand(int m, int K, const float* S, const int32_t* kmin, float* T,
                             int64_t ldt, hipStream_t s) {
  const dim3 grid((m + kLotExpTJ - 1) / kLotExpTJ, (m + kLotExpTI - 1) / kLotExpTI, K);
  const bool vec = (m % 4 == 0) && (ldt % 4 == 0) && ((uintptr_t)T % 16 == 0);
  if (vec) hipLaunchKernelGGL(lot_expand_kernel<true>, grid, dim3(256), 0, s, m, K, S, kmin, T, ldt);
  else hipLaunchKernelGGL(lot_expand_kernel<false>, grid, dim3(256), 0, s, m, K, S, kmin, T, ldt);
  return hipGetLastError();
}

}  // namespace csot
