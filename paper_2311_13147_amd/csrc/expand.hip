// Expansion of the reduced solution to the full block-circulant plan.
//
//   T[r m + i, c m + j] = exp((f_i + g_j - C_{ij,(c - r) mod K}) / eps)
//
// Lemma 1 (eq. blkstr_optimal_solution) says an optimal plan has the same block-circulant
// structure as the cost, and eq. optimality_condition with phi*(y) = eps exp(y/eps) gives the
// entries T_ijk of block k from the dual potentials (Alg. 2, last steps).  Each thread
// evaluates four consecutive entries of block k once (4 exponentials) and stores them to the
// K places that block k occupies, one per block-row: n*n*4 bytes written for K*m*m
// exponentials, so the kernel is bound by HBM write bandwidth.  Stores are non-temporal.
#include "common.hpp"
#include "launch.hpp"

namespace csot {

constexpr int kExpTJ = 256;  // j per block row segment (64 lanes x float4)
constexpr int kExpTI = 4;    // i per block (one wave each)

template <int DIM>
__device__ __forceinline__ float block_cost(const Geom& g, int i, int k, int j) {
  if constexpr (DIM == 0) {
    return g.C[(int64_t)i * g.ldc + (int64_t)k * g.m + j];
  } else {
    const int J = k * g.m + j;
    float c = 0.0f;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const float df = g.x[(int64_t)i * DIM + d] - g.y[(int64_t)J * DIM + d];
      c = fmaf(df, df, c);
    }
    return c;
  }
}

template <int DIM, bool VEC>
__global__ void __launch_bounds__(256)
    expand_kernel(Geom g, const float* __restrict__ f, const float* __restrict__ gp,
                  float* __restrict__ T, int64_t ldt, float s2) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.y * kExpTI + wv;
  const int k = blockIdx.z;
  const int j0 = blockIdx.x * kExpTJ + lane * 4;
  if (i >= g.m || j0 >= g.m) return;
  const float fi = f[i];
  float v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = j0 + q;
    v[q] = j < g.m ? exp2_fast((fi + gp[j] - block_cost<DIM>(g, i, k, j)) * s2) : 0.0f;
  }
  for (int r = 0; r < g.K; ++r) {
    const int c = r + k < g.K ? r + k : r + k - g.K;
    float* dst = T + (int64_t)(r * g.m + i) * ldt + (int64_t)c * g.m + j0;
    if constexpr (VEC) {
      typedef float v4f __attribute__((ext_vector_type(4)));
      const v4f val = {v[0], v[1], v[2], v[3]};
      __builtin_nontemporal_store(val, reinterpret_cast<v4f*>(dst));
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (j0 + q < g.m) __builtin_nontemporal_store(v[q], dst + q);
    }
  }
}

hipError_t launch_expand(const Geom& g, const float* f, const float* gp, float* T, int64_t ldt,
                         hipStream_t s) {
  const dim3 grid((g.m + kExpTJ - 1) / kExpTJ, (g.m + kExpTI - 1) / kExpTI, g.K);
  const bool vec = (g.m % 4 == 0) && (ldt % 4 == 0) && ((uintptr_t)T % 16 == 0);
  const float s2 = (float)(kLog2eD / g.eps);
#define CSOT_EXP(D)                                                                            \
  if (vec) hipLaunchKernelGGL((expand_kernel<D, true>), grid, dim3(256), 0, s, g, f, gp, T, ldt, s2); \
  else hipLaunchKernelGGL((expand_kernel<D, false>), grid, dim3(256), 0, s, g, f, gp, T, ldt, s2);
  switch (g.dim) {
    case 0: CSOT_EXP(0) break;
    case 2: CSOT_EXP(2) break;
    case 3: CSOT_EXP(3) break;
    default: return hipErrorInvalidValue;
  }
#undef CSOT_EXP
  return hipGetLastError();
}

}  // namespace csot
