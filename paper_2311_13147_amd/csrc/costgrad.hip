// Objective values, gradients and float64 marginal checks from dual potentials.
//
// Values (full problem; for reduced potentials the sums over (i, j, k) are multiplied by K,
// the 1/K identity of eq. problem_CROT):
//   P = sum T (C + eps (Z - 1)),  Z = (f + g - C) / eps,  T = exp(Z)   -- the primal of eq.
//       problem_ROT with the entropic regulariser evaluated without forming log T;
//   D = <f, a> + <g, b> - eps sum T                                    -- eq. dual_problem_cyclic_ROT;
//   <C, T>, sum T and the L2 marginal errors.
// Gradients (envelope theorem on the dual; exact at the optimum):
//   dC = T (for reduced potentials: the derivative with respect to block-row 0 of the cost,
//   each entry of which appears in all K block-rows: dC[i, k m + j] = K T_ijk);
//   da = f - mean(f);  db = g - mean(g);
//   dx_I = 2 sum_J T_IJ (x_I - y_J);  dy_J = 2 sum_I T_IJ (y_J - x_I).
// With reduced potentials T_IJ is the expanded plan, T[r m + i, c m + j] = T_{ij,(c-r) mod K}
// (Lemma 1), whose cost is block-row 0's; the gradient weights use the actual coordinates.
//
// Everything is organised as "passes": a wave owns four points of one side (rows for the row
// pass, columns for the column pass) and its lanes stride over all points of the other side,
// so every sum over the other side is a register accumulation plus one wave reduction -- no
// atomics.  For reduced potentials the other side is walked block by block, so the cyclic
// block index (c - r) mod K is computed once per block, not per entry.  Per-term arithmetic is
// float32 with one exponential per entry; sums of squares and scalars are float64.  The
// float64 marginal checks of the solvers use the same passes with float64 exponentials.
#include "common.hpp"
#include "launch.hpp"

namespace csot {

constexpr int kPassThreads = 256;
constexpr int kPassRT = 4;  // own points per workgroup, shared by its waves
constexpr int kPassWaves = kPassThreads / kWave;
constexpr int kPassPts = kPassRT;

template <int DIM>
__device__ __forceinline__ float pt_cost_f(const float* __restrict__ x, int I,
                                           const float* __restrict__ y, int J) {
  float c = 0.0f;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const float df = x[(int64_t)I * DIM + d] - y[(int64_t)J * DIM + d];
    c = fmaf(df, df, c);
  }
  return c;
}

struct PassOut {
  double* sums;   // [own points] sum over the other side of T (row or column sums)
  double* part;   // [blocks][3] P, <C,T>, mass partials (row pass) or nullptr
  float* grad;    // [own points, DIM] 2 sum T (own - other), or nullptr
  float* dC;      // row pass only: full [n, lddc] (= T); reduced block-row 0 [m, lddc]
                  // (dC[i, k m + j] = K T_ijk); or nullptr
  int64_t lddc;
};

// The inner loop of a pass when the workgroup's own points are all valid and, for reduced
// potentials, lie in one block: the cost's block index is then uniform per partner block and
// the flags (values and sums, plan entries, gradients) are compile-time, so the loop holds no
// branches.  VALS: row / column sums (and, in the row pass, P and <C, T>) -- for reduced
// potentials only block 0's points carry them (every block of the expanded plan holds the
// same values, Lemma 1).  DC: store the plan entries.  GRAD: coordinate gradients.
template <int DIM, bool RED, bool ROW, bool VALS, bool DC, bool GRAD>
__device__ __forceinline__ void pass_fast(const Geom& g, const float* __restrict__ f,
                                          const float* __restrict__ gp, float s2, float eps,
                                          const PassOut& out, int a0, int wv, int lane,
                                          const int (&ab)[kPassRT], const int (&ai)[kPassRT],
                                          const float (&po)[kPassRT][DIM],
                                          const float (&pot)[kPassRT],
                                          const float (&xc)[kPassRT][DIM],
                                          float (&tsum)[kPassRT], float (&gacc)[kPassRT][DIM],
                                          float (&vP)[kPassRT], float (&vC)[kPassRT]) {
  const int nblk = RED ? g.K : 1;
  const int bl = RED ? g.m : g.n;
  const float* othp = ROW ? g.y : g.x;
  for (int cb = 0; cb < nblk; ++cb) {
    int kk = 0;  // block of the cost: ROW (c - r) mod K with c = cb; COL (own c - r), r = cb
    if constexpr (RED) {
      kk = ROW ? cb - ab[0] : ab[0] - cb;
      if (kk < 0) kk += g.K;
    }
    // reduced column pass: the own column's block-row 0 partner y_{k m + j} is fixed per block
    float xq[kPassRT][DIM];
#pragma unroll
    for (int q = 0; q < kPassRT; ++q)
#pragma unroll
      for (int d = 0; d < DIM; ++d)
        xq[q][d] = !RED ? 0.0f : ROW ? xc[q][d] : g.y[((int64_t)kk * g.m + ai[q]) * DIM + d];
    // per partner b: the cost partner (reduced: block-row 0's point) and the actual partner
    const float* costp = RED ? (ROW ? g.y + (int64_t)kk * g.m * DIM : g.x) : othp;
    const float* gradp = othp + (int64_t)cb * bl * DIM;
    float* dcrow[kPassRT];
#pragma unroll
    for (int q = 0; q < kPassRT; ++q)
      dcrow[q] = !(DC && ROW) ? nullptr
                 : RED ? out.dC + (int64_t)ai[q] * out.lddc + (int64_t)kk * g.m
                       : out.dC + (int64_t)(a0 + q) * out.lddc;
#pragma unroll 2
    for (int b = lane + wv * kWave; b < bl; b += kPassThreads) {
      float pb[DIM], cp[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) pb[d] = gradp[(int64_t)b * DIM + d];
      if constexpr (RED) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) cp[d] = costp[(int64_t)b * DIM + d];
      }
      const float op = ROW ? gp[b] : f[b];  // reduced: index b of block 0; full: cb = 0
#pragma unroll
      for (int q = 0; q < kPassRT; ++q) {
        float df[DIM];
        float c = 0.0f;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          df[d] = po[q][d] - pb[d];
          if constexpr (RED) {
            const float e = ROW ? xq[q][d] - cp[d] : cp[d] - xq[q][d];
            c = fmaf(e, e, c);
          } else {
            c = fmaf(df[d], df[d], c);
          }
        }
        const float fg = pot[q] + op;
        const float T = exp2_fast((fg - c) * s2);
        if constexpr (VALS) {
          tsum[q] += T;
          if constexpr (ROW) {
            vP[q] = fmaf(T, fg - eps, vP[q]);  // T (C + eps (Z - 1)) = T (f + g - eps)
            vC[q] = fmaf(T, c, vC[q]);
          }
        }
        if constexpr (DC && ROW) dcrow[q][b] = RED ? (float)g.K * T : T;
        if constexpr (GRAD) {
#pragma unroll
          for (int d = 0; d < DIM; ++d) gacc[q][d] = fmaf(T, df[d], gacc[q][d]);
        }
      }
    }
  }
}

// One pass in float32 (values / gradients).  ROW: own = rows I (x), other = columns J (y).
// RED: potentials f, g have length m and the cost is block-row 0's.  `own_count` limits the
// own points (m when only block 0 is needed, n otherwise).
template <int DIM, bool RED, bool ROW>
__global__ void __launch_bounds__(kPassThreads)
    pass_kernel(Geom g, const float* __restrict__ f, const float* __restrict__ gp, float s2,
                float eps, int own_count, PassOut out) {
  // the workgroup's waves share its four own points and split the other side among them
  __shared__ double sh_d[kPassWaves][3][kPassRT];
  __shared__ float sh_g[kPassWaves][kPassRT][DIM > 0 ? DIM : 1];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int a0 = blockIdx.x * kPassRT;
  const float* ownp = ROW ? g.x : g.y;
  const float* othp = ROW ? g.y : g.x;
  float po[kPassRT][DIM > 0 ? DIM : 1];
  float pot[kPassRT];
  int ab[kPassRT], ai[kPassRT], ax[kPassRT];  // block, in-block and clamped global index
  float tsum[kPassRT], gacc[kPassRT][DIM > 0 ? DIM : 1];
  float vP[kPassRT], vC[kPassRT];
#pragma unroll
  for (int q = 0; q < kPassRT; ++q) {
    const int A = min(a0 + q, own_count - 1);
    ax[q] = A;
    ab[q] = A / g.m;
    ai[q] = A - ab[q] * g.m;
    if constexpr (DIM > 0) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) po[q][d] = ownp[(int64_t)A * DIM + d];
    }
    pot[q] = RED ? (ROW ? f[ai[q]] : gp[ai[q]]) : (ROW ? f[A] : gp[A]);
    tsum[q] = 0.0f;
    vP[q] = 0.0f;
    vC[q] = 0.0f;
#pragma unroll
    for (int d = 0; d < (DIM > 0 ? DIM : 1); ++d) gacc[q][d] = 0.0f;
  }
  const int nblk = RED ? g.K : 1;
  const int bl = RED ? g.m : g.n;
  // RED with coordinates: the cost uses block-row 0's points -- ROW: x_i (own, fixed) against
  // y_{k m + b}; COL: x_b (the partner itself) against y_{k m + j} (own, fixed per block)
  float xc[kPassRT][DIM > 0 ? DIM : 1];
  if constexpr (RED && ROW && DIM > 0) {
#pragma unroll
    for (int q = 0; q < kPassRT; ++q)
#pragma unroll
      for (int d = 0; d < DIM; ++d) xc[q][d] = g.x[(int64_t)ai[q] * DIM + d];
  }
  bool fast = false;
  if constexpr (DIM > 0) {
    if (a0 + kPassRT <= own_count && (!RED || ab[0] == ab[kPassRT - 1])) {
      fast = true;
      const bool vals = !RED || ab[0] == 0;
      const bool dc = ROW && out.dC != nullptr && vals;
      const bool gr = out.grad != nullptr;
#define CSOT_PF(V, D, G)                                                                    \
  pass_fast<DIM, RED, ROW, V, D, G>(g, f, gp, s2, eps, out, a0, wv, lane, ab, ai, po, pot, xc, \
                                    tsum, gacc, vP, vC)
      if (vals && dc) {
        if (gr) CSOT_PF(true, true, true); else CSOT_PF(true, true, false);
      } else if (vals) {
        if (gr) CSOT_PF(true, false, true); else CSOT_PF(true, false, false);
      } else {
        if (gr) CSOT_PF(false, false, true); else CSOT_PF(false, false, false);
      }
#undef CSOT_PF
    }
  }
  for (int cb = 0; cb < (fast ? 0 : nblk); ++cb) {
    int kk[kPassRT];
#pragma unroll
    for (int q = 0; q < kPassRT; ++q) {
      // block of the cost: ROW: (c - r) mod K with c = cb, r = own block; COL: (own c - r)
      int k = ROW ? cb - ab[q] : ab[q] - cb;
      kk[q] = k < 0 ? k + g.K : k;
    }
    if constexpr (RED && !ROW && DIM > 0) {
#pragma unroll
      for (int q = 0; q < kPassRT; ++q)
#pragma unroll
        for (int d = 0; d < DIM; ++d) xc[q][d] = g.y[((int64_t)kk[q] * g.m + ai[q]) * DIM + d];
    }
    // the own points of a wave usually share one block: then one cost point serves all four
    const bool same_k = kk[0] == kk[kPassRT - 1] && kk[1] == kk[0] && kk[2] == kk[0];
#pragma unroll 2
    for (int b = lane + wv * kWave; b < bl; b += kPassThreads) {
      const int B = cb * bl + b;  // other point (global index)
      float pb[DIM > 0 ? DIM : 1];
      if constexpr (DIM > 0) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) pb[d] = othp[(int64_t)B * DIM + d];
      }
      float yc[DIM > 0 ? DIM : 1];  // RED ROW: y_{k m + b} of the common block
      if constexpr (RED && ROW && DIM > 0) {
        if (same_k) {
#pragma unroll
          for (int d = 0; d < DIM; ++d) yc[d] = g.y[((int64_t)kk[0] * g.m + b) * DIM + d];
        }
      }
      const float opot = RED ? (ROW ? gp[b] : f[b]) : (ROW ? gp[B] : f[B]);
#pragma unroll
      for (int q = 0; q < kPassRT; ++q) {
        float c;
        if constexpr (RED) {
          // block-row 0 cost between point i (row) and point k m + j (column)
          const int i = ROW ? ai[q] : b;
          const int j = ROW ? b : ai[q];
          if constexpr (DIM == 0) {
            c = g.C[(int64_t)i * g.ldc + (int64_t)kk[q] * g.m + j];
          } else {
            c = 0.0f;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
              float other;
              if constexpr (ROW) other = same_k ? yc[d] : g.y[((int64_t)kk[q] * g.m + b) * DIM + d];
              else other = g.x[(int64_t)b * DIM + d];
              const float df = (ROW ? xc[q][d] : other) - (ROW ? other : xc[q][d]);
              c = fmaf(df, df, c);
            }
          }
        } else {
          if constexpr (DIM == 0) {
            const int I = ROW ? ax[q] : B, J = ROW ? B : ax[q];
            c = g.C[(int64_t)I * g.ldc + J];
          } else {
            c = 0.0f;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
              const float df = po[q][d] - pb[d];
              c = fmaf(df, df, c);
            }
          }
        }
        const float fg = pot[q] + opot;
        const float T = exp2_fast((fg - c) * s2);
        // reduced potentials: every block-row (column) of the expanded plan holds the same
        // values (Lemma 1), so sums and values come from block 0's points alone (x K)
        if (!RED || ab[q] == 0) {
          tsum[q] += T;
          if constexpr (ROW) {
            // T (C + eps (Z - 1)) with Z = (f + g - C) / eps is T (f + g - eps)
            vP[q] = fmaf(T, fg - eps, vP[q]);
            vC[q] = fmaf(T, c, vC[q]);
          }
        }
        if constexpr (ROW) {
          if (out.dC && a0 + q < own_count) {
            if constexpr (RED) {
              if (ab[q] == 0)
                out.dC[(int64_t)ai[q] * out.lddc + (int64_t)kk[q] * g.m + b] = (float)g.K * T;
            } else {
              out.dC[(int64_t)(a0 + q) * out.lddc + B] = T;
            }
          }
        }
        if constexpr (DIM > 0) {
          if (out.grad) {
#pragma unroll
            for (int d = 0; d < DIM; ++d) gacc[q][d] = fmaf(T, po[q][d] - pb[d], gacc[q][d]);
          }
        }
      }
    }
  }
  // lanes, then the waves (fixed order) of each own point
#pragma unroll
  for (int q = 0; q < kPassRT; ++q) {
    const double ts = wave_sum_d((double)tsum[q]);
    const double P = ROW ? wave_sum_d((double)vP[q]) : 0.0;
    const double C = ROW ? wave_sum_d((double)vC[q]) : 0.0;
    if (lane == 0) { sh_d[wv][0][q] = ts; sh_d[wv][1][q] = P; sh_d[wv][2][q] = C; }
    if constexpr (DIM > 0) {
      if (out.grad) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const float v = wave_sum(gacc[q][d]);
          if (lane == 0) sh_g[wv][q][d] = v;
        }
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bp = 0.0, bc = 0.0, bm = 0.0;
    for (int q = 0; q < kPassRT; ++q) {
      if (a0 + q >= own_count) break;
      double ts = 0.0, P = 0.0, C = 0.0;
      for (int w = 0; w < kPassWaves; ++w) { ts += sh_d[w][0][q]; P += sh_d[w][1][q]; C += sh_d[w][2][q]; }
      out.sums[a0 + q] = ts;
      bp += P; bc += C; bm += ts;
      if constexpr (DIM > 0) {
        if (out.grad) {
          for (int d = 0; d < DIM; ++d) {
            float v = 0.0f;
            for (int w = 0; w < kPassWaves; ++w) v += sh_g[w][q][d];
            out.grad[(int64_t)(a0 + q) * DIM + d] = 2.0f * v;
          }
        }
      }
    }
    if (ROW && out.part) {
      out.part[3 * blockIdx.x + 0] = bp;
      out.part[3 * blockIdx.x + 1] = bc;
      out.part[3 * blockIdx.x + 2] = bm;
    }
  }
}

// ---- reduced potentials with coordinates: one exponential per (i, j, k) ------------------
// The expanded plan has K m^2 distinct entries T_ijk (Lemma 1), so each is evaluated once per
// pass.  Workgroup o < m is the row pass for block-0 row i = o: every lane takes partners j,
// loads y_{c m + j} for all blocks c, evaluates T_ijk for all k (cost of block-row 0,
// |x_i - y_{k m + j}|^2) and accumulates the row sum S_i, P and <C, T> from them, stores dC,
// and forms in float64
//   Y_i(r) = sum_{k, j} T_ijk y_{((r + k) mod K) m + j},   dx_{r m + i} = 2 (x_{r m + i} S_i - Y_i(r)),
// the gradient of every block's copy of row i (T[r m + i, c m + j] = T_{ij,(c-r) mod K}).
// Workgroup m + o is the column pass for column j = o: partners i, T_ijk for all k from
// x_i and the own y_{k m + j}, the column sum S'_j and
//   X_j(c) = sum_{k, i} T_ijk x_{((c - k) mod K) m + i},   dy_{c m + j} = 2 (y_{c m + j} S'_j - X_j(c)).
// The K^2 products per partner are float64 FMAs of the float32 plan entries and coordinates
// (exact products), and S is summed in float64, so x S - Y keeps full accuracy despite the
// cancellation: the result is the gradient of the float32-rounded plan.
constexpr int kAdjThreads = 256;
constexpr int kAdjWaves = kAdjThreads / kWave;

// K values the adjoint kernel is instantiated for (its K dim float64 sums and K plan entries
// per partner stay in registers up to K = 16); others use pass_kernel.
__host__ __device__ constexpr bool adj_supported(int K, int dim) {
  return (dim == 2 || dim == 3) && (K == 1 || K == 2 || K == 4 || K == 8 || K == 16);
}

// Per-point partials of the adjoint kernel (float64), one row of kAdjPart per block-0 index:
// row workgroup o: P, <C,T>, mass (sum T), (rowsum - alpha)^2, f alpha; column workgroup o:
// (colsum - beta)^2, g beta.
constexpr int kAdjPart = 8;

struct AdjOut {
  double* part;    // [m][kAdjPart]
  float* dx;       // [n, DIM] or nullptr
  float* dy;       // [n, DIM] or nullptr
  float* dC;       // [m, lddc]: dC[i, k m + j] = K T_ijk, or nullptr
  int64_t lddc;
  float* da;       // [n] or nullptr: f tiled, mean-centred
  float* db;       // [n] or nullptr
};

template <int DIM, int KT, bool ROW, int NV>
__device__ __forceinline__ void adj_accumulate(const float (&pt)[KT][DIM], const double (&T64)[KT],
                                               double (&acc)[NV]) {
#pragma unroll
  for (int a = 0; a < KT; ++a) {
    double pv[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) pv[d] = (double)pt[a][d];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      const int t = ROW ? (a - k + KT) % KT : (a + k) % KT;  // output block
#pragma unroll
      for (int d = 0; d < DIM; ++d) acc[t * DIM + d] = fma(T64[k], pv[d], acc[t * DIM + d]);
    }
  }
}

// Float64 sum over the workgroup (fixed order: waves, then lanes), every thread receiving it.
__device__ __forceinline__ double adj_block_sum(double v, double* sh) {
  v = wave_sum_all_d(v);
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kAdjWaves; ++w) t += sh[w];
  return t;
}

// One own point o of block 0: row i = o (ROW) or column j = o.
template <int DIM, int KT, bool ROW>
__device__ __forceinline__ void adj_body(const Geom& g, const float* __restrict__ f,
                                         const float* __restrict__ gp, float s2, float eps,
                                         const AdjOut& out, int o) {
  constexpr int NA = KT * DIM;               // gradient sums per own point: (block, component)
  constexpr int SH = ilog2_ceil(NA);         // reduce-scatter over 2^SH values
  constexpr int NV = 1 << SH;
  __shared__ double sh_acc[kAdjWaves][NV];
  __shared__ double sh_red[kAdjWaves];
  __shared__ float own_pts[ROW ? 1 : KT][DIM];  // column pass: y_{k m + j} of the own column
  const int m = g.m;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  float* __restrict__ grad_out = ROW ? out.dx : out.dy;
  const bool grad = grad_out != nullptr;
  const bool dc = ROW && out.dC != nullptr;
  const float* __restrict__ x = g.x;
  const float* __restrict__ y = g.y;

  float xo[DIM];  // row pass: x_i (block 0)
  if constexpr (ROW) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) xo[d] = x[(int64_t)o * DIM + d];
  } else {
    if (threadIdx.x < NA) {
      const int k = threadIdx.x / DIM, d = threadIdx.x - k * DIM;
      own_pts[k][d] = y[((int64_t)k * m + o) * DIM + d];
    }
    __syncthreads();
  }
  const float po = ROW ? f[o] : gp[o];

  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  double S = 0.0;
  float vP = 0.0f, vC = 0.0f;

#pragma unroll 1
  for (int p = threadIdx.x; p < m; p += kAdjThreads) {
    // the partner's coordinates in every block: row pass y_{c m + j}, column pass x_{r m + i}
    float pt[KT][DIM];
    const float* __restrict__ src = ROW ? y : x;
#pragma unroll
    for (int c = 0; c < KT; ++c)
#pragma unroll
      for (int d = 0; d < DIM; ++d) pt[c][d] = src[((int64_t)c * m + p) * DIM + d];
    const float fg = po + (ROW ? gp[p] : f[p]);
    double T64[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      // block-row 0 cost |x_i - y_{k m + j}|^2: row pass x_i own, y_{k m + j} = pt[k];
      // column pass x_i = pt[0], y_{k m + j} own
      float c = 0.0f;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const float e = ROW ? xo[d] - pt[k][d] : pt[0][d] - own_pts[ROW ? 0 : k][d];
        c = fmaf(e, e, c);
      }
      const float T = exp2_fast((fg - c) * s2);
      T64[k] = (double)T;
      S += T64[k];
      if constexpr (ROW) {
        vP = fmaf(T, fg - eps, vP);  // T (C + eps (Z - 1)) = T (f + g - eps)
        vC = fmaf(T, c, vC);
        if (dc) out.dC[(int64_t)o * out.lddc + (int64_t)k * m + p] = (float)g.K * T;
      }
    }
    // row: Y(r) += T_k y_{((r + k) mod K)}: pt[a] (block a = r + k) feeds output r = a - k;
    // column: X(c) += T_k x_{((c - k) mod K)}: pt[a] (block a = c - k) feeds output c = a + k
    if (grad) adj_accumulate<DIM, KT, ROW>(pt, T64, acc);
  }

  // the own point's folded marginal (mean over the K blocks) and the potential's mean (for
  // da / db), both summed by every workgroup in the same order
  const float* __restrict__ marg = ROW ? g.a : g.b;
  const float* __restrict__ pot = ROW ? f : gp;
  double mv = threadIdx.x < KT ? (double)marg[(int64_t)threadIdx.x * m + o] : 0.0;
  double ps = 0.0;
  for (int p = threadIdx.x; p < m; p += kAdjThreads) ps += (double)pot[p];
  const double tS = adj_block_sum(S, sh_red);
  const double tP = ROW ? adj_block_sum((double)vP, sh_red) : 0.0;
  const double tC = ROW ? adj_block_sum((double)vC, sh_red) : 0.0;
  const double marg_o = adj_block_sum(mv, sh_red) / KT;
  const double pmean = adj_block_sum(ps, sh_red) / m;
  if (grad) {
    wave_reduce_scatter_d<SH>(acc, lane);
    if ((lane & ((64 >> SH) - 1)) == 0) sh_acc[wv][lane >> (6 - SH)] = acc[0];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* pr = out.part + (int64_t)o * kAdjPart;
    const double dr = tS - marg_o;
    if constexpr (ROW) {
      pr[0] = tP;
      pr[1] = tC;
      pr[2] = tS;
      pr[3] = dr * dr;
      pr[4] = (double)po * marg_o;
    } else {
      pr[5] = dr * dr;
      pr[6] = (double)po * marg_o;
    }
  }
  float* __restrict__ dpot = ROW ? out.da : out.db;
  if (dpot && threadIdx.x < KT) dpot[(int64_t)threadIdx.x * m + o] = (float)((double)po - pmean);
  if (grad && threadIdx.x < NA) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kAdjWaves; ++w) v += sh_acc[w][threadIdx.x];
    const int blk = threadIdx.x / DIM, d = threadIdx.x - blk * DIM;
    const int64_t P = (int64_t)blk * m + o;  // the own point's copy in block blk
    const double own = (double)(ROW ? x : y)[P * DIM + d];
    grad_out[P * DIM + d] = (float)(2.0 * (own * tS - v));
  }
}

// Workgroups [0, m): rows; [m, 2 m): columns.
template <int DIM, int KT>
__global__ void __launch_bounds__(kAdjThreads)
    red_adjoint_kernel(Geom g, const float* __restrict__ f, const float* __restrict__ gp,
                       float s2, float eps, AdjOut out) {
  const int b = blockIdx.x;
  if (b < g.m) adj_body<DIM, KT, true>(g, f, gp, s2, eps, out, b);
  else adj_body<DIM, KT, false>(g, f, gp, s2, eps, out, b - g.m);
}

// The scalars of the full problem from the per-point partials: P, D, <C,T>, both marginal
// errors and the mass, each a K-multiple of the reduced sum (eq. problem_CROT).
__global__ void __launch_bounds__(kAdjThreads)
    red_finalize_kernel(int m, int K, double eps, const double* __restrict__ part,
                        double* __restrict__ out) {
  __shared__ double sh[kAdjWaves];
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int o = threadIdx.x; o < m; o += kAdjThreads) {
#pragma unroll
    for (int q = 0; q < 7; ++q) v[q] += part[(int64_t)o * kAdjPart + q];
  }
#pragma unroll
  for (int q = 0; q < 7; ++q) v[q] = adj_block_sum(v[q], sh);
  if (threadIdx.x == 0) {
    const double Kd = (double)K;
    out[0] = Kd * v[0];
    out[1] = Kd * (v[4] + v[6]) - eps * Kd * v[2];
    out[2] = Kd * v[1];
    out[3] = sqrt(Kd * v[3]);
    out[4] = sqrt(Kd * v[5]);
    out[5] = Kd * v[2];
    out[6] = 0.0;
    out[7] = 0.0;
  }
}

// float64 marginal sums.  MODE 0: reduced, exponent logK_ij + (f_i + g_j)/eps over [0, m);
// MODE 1: full from coordinates (DIM) or dense C, exponent (f_I + g_J - C_IJ)/eps.
template <int MODE, int DIM, bool ROW>
__global__ void __launch_bounds__(kPassThreads)
    check_pass_kernel(Geom g, const float* __restrict__ logK, const float* __restrict__ f,
                      const float* __restrict__ gp, int N, double* __restrict__ sums) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int a = blockIdx.x * (kPassThreads / kWave) + wv;
  if (a >= N) return;
  const double ie = 1.0 / g.eps;
  const double pa = ROW ? (double)f[a] : (double)gp[a];
  double s = 0.0;
  for (int b = lane; b < N; b += kWave) {
    const double pb = ROW ? (double)gp[b] : (double)f[b];
    const int I = ROW ? a : b, J = ROW ? b : a;
    double z;
    if constexpr (MODE == 0) {
      z = (double)logK[(int64_t)I * N + J] + (pa + pb) * ie;
    } else {
      double c;
      if constexpr (DIM == 0) {
        c = (double)g.C[(int64_t)I * g.ldc + J];
      } else {
        c = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
          const double df = (double)g.x[(int64_t)I * DIM + d] - (double)g.y[(int64_t)J * DIM + d];
          c += df * df;
        }
      }
      z = (pa + pb - c) * ie;
    }
    s += exp(z);
  }
  s = wave_sum_d(s);
  if (lane == 0) sums[a] = s;
}

// norms of (rowsum - ra), (colsum - rb) over N entries; `scale` (K for reduced sums) turns
// them into full-space norms.
// One workgroup of kFinThreads threads; loops keep four iterations' loads in flight.
constexpr int kFinThreads = 1024;

__global__ void __launch_bounds__(kFinThreads)
    check_finalize_kernel(int N, double scale, const double* __restrict__ rowsum,
                          const double* __restrict__ colsum, const float* __restrict__ ra,
                          const float* __restrict__ rb, double* __restrict__ dstats) {
  __shared__ double red[kFinThreads / kWave];
  double er = 0.0, ec = 0.0;
#pragma unroll 4
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const double dr = rowsum[i] - (double)ra[i], dc = colsum[i] - (double)rb[i];
    er += dr * dr;
    ec += dc * dc;
  }
  er = block_sum_d(er, red);
  ec = block_sum_d(ec, red);
  if (threadIdx.x == 0) {
    dstats[2] = sqrt(scale * er);
    dstats[3] = sqrt(scale * ec);
  }
}

// ---- finalize: scalars, marginal errors, da / db ----------------------------------------
__global__ void __launch_bounds__(kFinThreads)
    finalize_kernel(Geom g, int red_mode, double scale, const float* __restrict__ f,
                    const float* __restrict__ gp, const double* __restrict__ part, int nparts,
                    const double* __restrict__ rowsum, const double* __restrict__ colsum,
                    double* __restrict__ out, float* __restrict__ da, float* __restrict__ db) {
  const int N = red_mode ? g.m : g.n;
  const double K = red_mode ? (double)g.K : 1.0;
  double P = 0.0, CT = 0.0, mass = 0.0;
#pragma unroll 4
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
    P += part[3 * b];
    CT += part[3 * b + 1];
    mass += part[3 * b + 2];
  }
  double fa = 0.0, gb = 0.0, er = 0.0, ec = 0.0, fs = 0.0, gs = 0.0;
#pragma unroll 4
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    double ai, bi;
    if (red_mode) {
      ai = 0.0;
      bi = 0.0;
#pragma unroll 8
      for (int r = 0; r < g.K; ++r) {  // eight blocks' loads in flight
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
  // the nine block sums in one pass: interleaved lane shuffles, one LDS round
  double v[9] = {P, CT, mass, fa, gb, er, ec, fs, gs};
  {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    for (int o = kWave / 2; o > 0; o >>= 1) {
#pragma unroll
      for (int k = 0; k < 9; ++k) v[k] += __shfl_xor(v[k], o, kWave);
    }
    __shared__ double sums9[kFinThreads / kWave][9];
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < 9; ++k) sums9[wid][k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      double t = 0.0;
      for (int w = 0; w < kFinThreads / kWave; ++w) t += sums9[w][k];
      v[k] = t;
    }
  }
  P = v[0]; CT = v[1]; mass = v[2]; fa = v[3]; gb = v[4]; er = v[5]; ec = v[6]; fs = v[7];
  gs = v[8];
  if (threadIdx.x == 0) {
    out[0] = scale * P;
    out[1] = K * (fa + gb) - g.eps * scale * mass;
    out[2] = scale * CT;
    out[3] = sqrt(K * er);
    out[4] = sqrt(K * ec);
    out[5] = scale * mass;
    out[6] = 0.0;
    out[7] = 0.0;
  }
  const double fm = fs / N, gm = gs / N;
#pragma unroll 4
  for (int I = threadIdx.x; I < g.n; I += blockDim.x) {
    const int i = red_mode ? I % g.m : I;
    if (da) da[I] = (float)((double)f[i] - fm);
    if (db) db[I] = (float)((double)gp[i] - gm);
  }
}

// ---- host ------------------------------------------------------------------------------
static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

static int pass_blocks(int count) { return (count + kPassPts - 1) / kPassPts; }

size_t costgrad_ws_bytes(const Geom& g) {
  // row / column sums [n] each, then the per-workgroup partials: pass_blocks(n) groups of the
  // pass kernels or m rows of the adjoint kernel
  const size_t parts = 3 * (size_t)pass_blocks(g.n) > (size_t)kAdjPart * (g.n / g.K)
                           ? 3 * (size_t)pass_blocks(g.n)
                           : (size_t)kAdjPart * (g.n / g.K);
  return 2 * align256(sizeof(double) * g.n) + align256(sizeof(double) * parts);
}

template <int DIM>
static hipError_t launch_adjoint(const Geom& g, const float* f, const float* gp, float s2,
                                 float eps, const AdjOut& o, hipStream_t s) {
  const dim3 grid(2 * g.m), blk(kAdjThreads);
#define CSOT_ADJ(KT) \
  hipLaunchKernelGGL((red_adjoint_kernel<DIM, KT>), grid, blk, 0, s, g, f, gp, s2, eps, o)
  switch (g.K) {
    case 1: CSOT_ADJ(1); break;
    case 2: CSOT_ADJ(2); break;
    case 4: CSOT_ADJ(4); break;
    case 8: CSOT_ADJ(8); break;
    case 16: CSOT_ADJ(16); break;
    default: return hipErrorInvalidValue;
  }
#undef CSOT_ADJ
  return hipGetLastError();
}

template <int DIM>
static hipError_t launch_passes(const Geom& g, const float* f, const float* gp, int reduced,
                                float s2, float eps, int rows, int cols, PassOut ro,
                                PassOut co, hipStream_t s) {
  if (reduced) {
    hipLaunchKernelGGL((pass_kernel<DIM, true, true>), dim3(pass_blocks(rows)),
                       dim3(kPassThreads), 0, s, g, f, gp, s2, eps, rows, ro);
    hipLaunchKernelGGL((pass_kernel<DIM, true, false>), dim3(pass_blocks(cols)),
                       dim3(kPassThreads), 0, s, g, f, gp, s2, eps, cols, co);
  } else {
    hipLaunchKernelGGL((pass_kernel<DIM, false, true>), dim3(pass_blocks(rows)),
                       dim3(kPassThreads), 0, s, g, f, gp, s2, eps, rows, ro);
    hipLaunchKernelGGL((pass_kernel<DIM, false, false>), dim3(pass_blocks(cols)),
                       dim3(kPassThreads), 0, s, g, f, gp, s2, eps, cols, co);
  }
  return hipGetLastError();
}

hipError_t launch_cost_and_grad(const Geom& g, const float* f, const float* gp, int reduced,
                                double* out, float* dC, int64_t lddc, float* dx, float* dy,
                                float* da, float* db, void* ws, hipStream_t s) {
  char* base = static_cast<char*>(ws);
  double* rowsum = reinterpret_cast<double*>(base);
  double* colsum = reinterpret_cast<double*>(base + align256(sizeof(double) * g.n));
  double* part = reinterpret_cast<double*>(base + 2 * align256(sizeof(double) * g.n));
  // Reduced potentials: the values and marginal sums come from block 0's points only (K m^2
  // terms, scaled by K); the coordinate gradients need every point (n^2 terms).
  const float s2 = (float)(kLog2eD / g.eps);
  const float eps = (float)g.eps;
  const double scale = reduced ? (double)g.K : 1.0;
  hipError_t e;
  if (reduced && adj_supported(g.K, g.dim)) {
    AdjOut ao{part, dx, dy, dC, lddc, da, db};
    e = g.dim == 2 ? launch_adjoint<2>(g, f, gp, s2, eps, ao, s)
                   : launch_adjoint<3>(g, f, gp, s2, eps, ao, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(red_finalize_kernel, dim3(1), dim3(kAdjThreads), 0, s, g.m, g.K, g.eps,
                       part, out);
    return hipGetLastError();
  }
  const bool all_rows = !reduced || dx != nullptr;
  const bool all_cols = !reduced || dy != nullptr;
  const int rows = all_rows ? g.n : g.m;
  const int cols = all_cols ? g.n : g.m;
  PassOut ro{rowsum, part, dx, dC, lddc};
  PassOut co{colsum, nullptr, dy, nullptr, 0};
  switch (g.dim) {
    case 0: e = launch_passes<0>(g, f, gp, reduced, s2, eps, rows, cols, ro, co, s); break;
    case 2: e = launch_passes<2>(g, f, gp, reduced, s2, eps, rows, cols, ro, co, s); break;
    case 3: e = launch_passes<3>(g, f, gp, reduced, s2, eps, rows, cols, ro, co, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kFinThreads), 0, s, g, reduced, scale, f, gp, part,
                     pass_blocks(rows), rowsum, colsum, out, da, db);
  return hipGetLastError();
}

// float64 marginal check used by the solvers.  reduced: potentials [m], logK, folded
// marginals ra, rb [m]; full: potentials [n], cost from g, ra = a, rb = b.  `sums` holds
// 2 N doubles of scratch.
hipError_t launch_check(const Geom& g, int reduced, const float* logK, const float* f,
                        const float* gp, const float* ra, const float* rb, double* sums,
                        double* dstats, hipStream_t s) {
  const int N = reduced ? g.m : g.n;
  double* rowsum = sums;
  double* colsum = sums + N;
  const dim3 grid((N + kPassThreads / kWave - 1) / (kPassThreads / kWave));
  const dim3 blk(kPassThreads);
  if (reduced) {
    hipLaunchKernelGGL((check_pass_kernel<0, 2, true>), grid, blk, 0, s, g, logK, f, gp, N, rowsum);
    hipLaunchKernelGGL((check_pass_kernel<0, 2, false>), grid, blk, 0, s, g, logK, f, gp, N, colsum);
  } else {
    switch (g.dim) {
      case 0:
        hipLaunchKernelGGL((check_pass_kernel<1, 0, true>), grid, blk, 0, s, g, logK, f, gp, N, rowsum);
        hipLaunchKernelGGL((check_pass_kernel<1, 0, false>), grid, blk, 0, s, g, logK, f, gp, N, colsum);
        break;
      case 2:
        hipLaunchKernelGGL((check_pass_kernel<1, 2, true>), grid, blk, 0, s, g, logK, f, gp, N, rowsum);
        hipLaunchKernelGGL((check_pass_kernel<1, 2, false>), grid, blk, 0, s, g, logK, f, gp, N, colsum);
        break;
      case 3:
        hipLaunchKernelGGL((check_pass_kernel<1, 3, true>), grid, blk, 0, s, g, logK, f, gp, N, rowsum);
        hipLaunchKernelGGL((check_pass_kernel<1, 3, false>), grid, blk, 0, s, g, logK, f, gp, N, colsum);
        break;
      default: return hipErrorInvalidValue;
    }
  }
  hipLaunchKernelGGL(check_finalize_kernel, dim3(1), dim3(kFinThreads), 0, s, N,
                     reduced ? (double)g.K : 1.0, rowsum, colsum, ra, rb, dstats);
  return hipGetLastError();
}

}  // namespace csot
