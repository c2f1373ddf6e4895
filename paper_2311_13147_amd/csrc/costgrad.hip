// Objective values and gradients of entropic OT from the (converged) dual potentials.
//
// Values (full problem; for reduced potentials the sums over (i, j, k) are multiplied by K,
// the 1/K identity of eq. problem_CROT):
//   P = sum T (C + eps (Z - 1)),  Z = (f + g - C) / eps,  T = exp(Z)   -- the primal of eq.
//       problem_ROT with the entropic regulariser evaluated without forming log T;
//   D = <f, a> + <g, b> - eps sum T                                    -- eq. dual_problem_cyclic_ROT;
//   <C, T>, sum T and the L2 marginal errors (row / column sums accumulated in float64).
// Gradients (envelope theorem on the dual; exact at the optimum):
//   dC = T;  da = f - mean(f);  db = g - mean(g);
//   dx_I = 2 sum_J T_IJ (x_I - y_J);  dy_J = 2 sum_I T_IJ (y_J - x_I).
// With reduced potentials T_IJ is the expanded plan, T[r m + i, c m + j] = T_{ij,(c-r) mod K},
// whose cost is block-row 0's; the gradient weights use the actual coordinates of I and J.
//
// Per-term arithmetic is float32 (one exponential per entry); scalar sums are float64.
#include "common.hpp"
#include "launch.hpp"

namespace csot {

constexpr int kCgTJ = 64;
constexpr int kCgTI = 4;

template <int DIM>
__device__ __forceinline__ float cost_pts(const float* __restrict__ x, int I,
                                          const float* __restrict__ y, int J) {
  float c = 0.0f;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const float df = x[(int64_t)I * DIM + d] - y[(int64_t)J * DIM + d];
    c = fmaf(df, df, c);
  }
  return c;
}

// ---- values, dC, row / column sums ------------------------------------------------------
// reduced: thread (i, j) of block k = blockIdx.z (cost of block-row 0);
// full:    thread (I, J), blockIdx.z == 0.
template <int DIM, bool RED>
__global__ void __launch_bounds__(kCgTJ* kCgTI)
    values_kernel(Geom g, const float* __restrict__ f, const float* __restrict__ gp, float s2,
                  float eps, float* __restrict__ dC, int64_t lddc,
                  double* __restrict__ part, double* __restrict__ rowsum,
                  double* __restrict__ colsum) {
  __shared__ double red[8];
  __shared__ double cacc[kCgTI][kCgTJ];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int N = RED ? g.m : g.n;
  const int j = blockIdx.x * kCgTJ + lane;
  const int i = blockIdx.y * kCgTI + wv;
  const int k = blockIdx.z;
  double P = 0.0, CT = 0.0, mass = 0.0, T64 = 0.0;
  if (i < N && j < N) {
    float c;
    if constexpr (RED) {
      if constexpr (DIM == 0) c = g.C[(int64_t)i * g.ldc + (int64_t)k * g.m + j];
      else c = cost_pts<DIM>(g.x, i, g.y, k * g.m + j);
    } else {
      if constexpr (DIM == 0) c = g.C[(int64_t)i * g.ldc + j];
      else c = cost_pts<DIM>(g.x, i, g.y, j);
    }
    const float fg = f[i] + gp[j];
    const float z = (fg - c) / eps;
    const float T = exp2_fast((fg - c) * s2);
    P = (double)(T * (c + eps * (z - 1.0f)));
    CT = (double)(T * c);
    mass = (double)T;
    T64 = (double)T;
    if (dC) {
      if constexpr (RED) dC[((int64_t)k * g.m + i) * g.m + j] = T;
      else dC[(int64_t)i * lddc + j] = T;
    }
  }
  // row sums: reduce across the wave; column sums: across the 4 waves
  const double rs = wave_sum_d(T64);
  if (lane == 0 && i < N) atomicAdd(&rowsum[i], rs);
  cacc[wv][lane] = T64;
  __syncthreads();
  if (wv == 0 && j < N)
    atomicAdd(&colsum[j], cacc[0][lane] + cacc[1][lane] + cacc[2][lane] + cacc[3][lane]);
  P = block_sum_d(P, red);
  CT = block_sum_d(CT, red);
  mass = block_sum_d(mass, red);
  if (threadIdx.x == 0) {
    const int64_t b = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    part[3 * b + 0] = P;
    part[3 * b + 1] = CT;
    part[3 * b + 2] = mass;
  }
}

// ---- coordinate gradients -----------------------------------------------------------------
// Each wave owns 4 points of the "own" side (x for dx, y for dy); lanes stride over the other
// side.  OWN_X: own = x (rows I), other = y (columns J); else own = y, other = x.
template <int DIM, bool RED, bool OWN_X>
__global__ void __launch_bounds__(256)
    coord_grad_kernel(Geom g, const float* __restrict__ f, const float* __restrict__ gp,
                      float s2, float* __restrict__ out) {
  constexpr int RT = 4;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int own0 = (blockIdx.x * 4 + wv) * RT;
  const float* ownp = OWN_X ? g.x : g.y;
  const float* othp = OWN_X ? g.y : g.x;
  float acc[RT][DIM];
  float po[RT][DIM];
#pragma unroll
  for (int q = 0; q < RT; ++q) {
    const int A = min(own0 + q, g.n - 1);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      acc[q][d] = 0.0f;
      po[q][d] = ownp[(int64_t)A * DIM + d];
    }
  }
  for (int B = lane; B < g.n; B += 64) {
    float pb[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) pb[d] = othp[(int64_t)B * DIM + d];
#pragma unroll
    for (int q = 0; q < RT; ++q) {
      const int A = min(own0 + q, g.n - 1);
      const int I = OWN_X ? A : B;  // row index of the plan entry
      const int J = OWN_X ? B : A;  // column index
      float c, fg;
      if constexpr (RED) {
        const int r = I / g.m, i = I - r * g.m, cb = J / g.m, j = J - cb * g.m;
        int kk = cb - r;
        if (kk < 0) kk += g.K;
        c = cost_pts<DIM>(g.x, i, g.y, kk * g.m + j);
        fg = f[i] + gp[j];
      } else {
        c = 0.0f;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const float df = po[q][d] - pb[d];
          c = fmaf(df, df, c);
        }
        fg = f[I] + gp[J];
      }
      const float T = exp2_fast((fg - c) * s2);
#pragma unroll
      for (int d = 0; d < DIM; ++d) acc[q][d] = fmaf(T, po[q][d] - pb[d], acc[q][d]);
    }
  }
#pragma unroll
  for (int q = 0; q < RT; ++q) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const float v = wave_sum(acc[q][d]);
      if (lane == 0 && own0 + q < g.n) out[(int64_t)(own0 + q) * DIM + d] = 2.0f * v;
    }
  }
}

// ---- finalize: scalars, marginal errors, da / db ----------------------------------------
__global__ void __launch_bounds__(256)
    finalize_kernel(Geom g, int red_mode, const float* __restrict__ f,
                    const float* __restrict__ gp, const double* __restrict__ part,
                    int64_t nparts, const double* __restrict__ rowsum,
                    const double* __restrict__ colsum, double* __restrict__ out,
                    float* __restrict__ da, float* __restrict__ db) {
  __shared__ double red[8];
  const int N = red_mode ? g.m : g.n;
  const double scale = red_mode ? (double)g.K : 1.0;
  double P = 0.0, CT = 0.0, mass = 0.0;
  for (int64_t b = threadIdx.x; b < nparts; b += blockDim.x) {
    P += part[3 * b];
    CT += part[3 * b + 1];
    mass += part[3 * b + 2];
  }
  P = block_sum_d(P, red);
  CT = block_sum_d(CT, red);
  mass = block_sum_d(mass, red);
  double fa = 0.0, gb = 0.0, er = 0.0, ec = 0.0, fs = 0.0, gs = 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    double ai, bi;
    if (red_mode) {
      ai = 0.0;
      bi = 0.0;
      for (int r = 0; r < g.K; ++r) {
        ai += (double)g.a[(int64_t)r * g.m + i];
        bi += (double)g.b[(int64_t)r * g.m + i];
      }
      ai /= g.K;
      bi /= g.K;
    } else {
      ai = g.a[i];
      bi = g.b[i];
    }
    fa += (double)f[i] * ai;
    gb += (double)gp[i] * bi;
    const double dr = rowsum[i] - ai, dc = colsum[i] - bi;
    er += dr * dr;
    ec += dc * dc;
    fs += f[i];
    gs += gp[i];
  }
  fa = block_sum_d(fa, red);
  gb = block_sum_d(gb, red);
  er = block_sum_d(er, red);
  ec = block_sum_d(ec, red);
  fs = block_sum_d(fs, red);
  gs = block_sum_d(gs, red);
  if (threadIdx.x == 0) {
    out[0] = scale * P;
    out[1] = scale * (fa + gb) - g.eps * scale * mass;
    out[2] = scale * CT;
    out[3] = sqrt(scale * er);
    out[4] = sqrt(scale * ec);
    out[5] = scale * mass;
    out[6] = 0.0;
    out[7] = 0.0;
  }
  const double fm = fs / N, gm = gs / N;
  for (int I = threadIdx.x; I < g.n; I += blockDim.x) {
    const int i = red_mode ? I % g.m : I;
    if (da) da[I] = (float)((double)f[i] - fm);
    if (db) db[I] = (float)((double)gp[i] - gm);
  }
}

__global__ void zero_d_kernel(double* p, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// ---- host ------------------------------------------------------------------------------
static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

static int64_t values_blocks(const Geom& g, int reduced, dim3* grid) {
  const int N = reduced ? g.m : g.n;
  *grid = dim3((N + kCgTJ - 1) / kCgTJ, (N + kCgTI - 1) / kCgTI, reduced ? g.K : 1);
  return (int64_t)grid->x * grid->y * grid->z;
}

size_t costgrad_ws_bytes(const Geom& g) {
  dim3 gr;
  const int64_t nb = values_blocks(g, 0, &gr);
  const int64_t nbr = values_blocks(g, 1, &gr);
  const int64_t nmax = nb > nbr ? nb : nbr;
  return 2 * align256(sizeof(double) * g.n) + align256(sizeof(double) * 3 * nmax);
}

hipError_t launch_cost_and_grad(const Geom& g, const float* f, const float* gp, int reduced,
                                double* out, float* dC, int64_t lddc, float* dx, float* dy,
                                float* da, float* db, void* ws, hipStream_t s) {
  char* base = static_cast<char*>(ws);
  const int N = reduced ? g.m : g.n;
  double* rowsum = reinterpret_cast<double*>(base);
  double* colsum = reinterpret_cast<double*>(base + align256(sizeof(double) * g.n));
  double* part = reinterpret_cast<double*>(base + 2 * align256(sizeof(double) * g.n));
  hipLaunchKernelGGL(zero_d_kernel, dim3(32), dim3(256), 0, s, rowsum,
                     (int64_t)(2 * align256(sizeof(double) * g.n) / sizeof(double)));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 grid;
  const int64_t nparts = values_blocks(g, reduced, &grid);
  const float s2 = (float)(kLog2eD / g.eps);
  const float epsf = (float)g.eps;
#define CSOT_VAL(D)                                                                             \
  if (reduced) hipLaunchKernelGGL((values_kernel<D, true>), grid, dim3(256), 0, s, g, f, gp, s2, epsf, dC, lddc, part, rowsum, colsum); \
  else hipLaunchKernelGGL((values_kernel<D, false>), grid, dim3(256), 0, s, g, f, gp, s2, epsf, dC, lddc, part, rowsum, colsum);
  switch (g.dim) {
    case 0: CSOT_VAL(0) break;
    case 2: CSOT_VAL(2) break;
    case 3: CSOT_VAL(3) break;
    default: return hipErrorInvalidValue;
  }
#undef CSOT_VAL
  if ((e = hipGetLastError()) != hipSuccess) return e;
  (void)N;
  if (g.dim > 0 && (dx || dy)) {
    const dim3 gg((g.n + 15) / 16);
#define CSOT_GR(D)                                                                                      \
  if (dx) { if (reduced) hipLaunchKernelGGL((coord_grad_kernel<D, true, true>), gg, dim3(256), 0, s, g, f, gp, s2, dx); \
            else hipLaunchKernelGGL((coord_grad_kernel<D, false, true>), gg, dim3(256), 0, s, g, f, gp, s2, dx); } \
  if (dy) { if (reduced) hipLaunchKernelGGL((coord_grad_kernel<D, true, false>), gg, dim3(256), 0, s, g, f, gp, s2, dy); \
            else hipLaunchKernelGGL((coord_grad_kernel<D, false, false>), gg, dim3(256), 0, s, g, f, gp, s2, dy); }
    if (g.dim == 2) { CSOT_GR(2) } else { CSOT_GR(3) }
#undef CSOT_GR
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, s, g, reduced, f, gp, part, nparts,
                     rowsum, colsum, out, da, db);
  return hipGetLastError();
}

}  // namespace csot
