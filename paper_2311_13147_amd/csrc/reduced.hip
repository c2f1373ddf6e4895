// Cyclic Sinkhorn on the folded m x m problem (Alg. 2), one persistent cooperative launch.
//
// Log-domain updates in base 2 (F = f log2(e) / eps, G = g log2(e) / eps, L = logK log2(e)):
//   row    (eq. optimal_f_sinkhorn_logdomain):  F_i = log2 alpha_i - LSE2_j(L_ij + G_j)
//   column (log of eq. optimal_sinkhorn):       G_j = log2 beta_j  - LSE2_i(L_ij + F_i)
// starting from G = 0 (q = 1, Alg. 2 initialisation) or a warm start.
//
// Work split: workgroup w owns rows [w R, w R + R) and columns [w R, w R + R).  It keeps its
// row slab of L and its column slab (a transposed copy) in LDS for the whole solve, so an
// iteration reads no matrix data from memory: only the other potential (m floats) is
// exchanged through global memory between two device-wide barriers per iteration.
//
// Convergence (a reading of "until convergence"): the row residual of the plan after
// iteration t-1 falls out of the row update of iteration t for free,
//   r_i = alpha_i (2^(F_i^{t-1} - F_i^t) - 1),
// because the row sums of that plan are alpha_i 2^(F^{t-1} - F^t).  Per-workgroup partial
// sums of r_i^2 are combined after the first barrier in a fixed order by every workgroup,
// so all take the same stop decision; the returned state is (F^{t-1}, G^{t-1}).  The
// full-space norm is sqrt(K) ||r||_2 (every block-row of the expanded plan has these sums).
//
// A separate check kernel recomputes both marginal errors in float64 from the returned f, g.
#include "common.hpp"
#include "launch.hpp"

namespace csot {

constexpr int kRedThreads = 256;
constexpr int kRedLPR = 16;            // lanes cooperating on one row / column
constexpr int kRedChunk = 4 * kRedLPR; // elements covered by one float4 sweep of a group
constexpr int kMaxLds = 150 * 1024;

struct RedParams {
  int m, mp, K, W, R, max_iter, warm;
  float s2;        // log2(e) / eps
  float to_nat;    // eps ln 2
  double tol2;     // tol^2 / K  (compared with sum r_i^2)
  const float* logK;
  const float* alpha;
  const float* beta;
  float* f_out;
  float* g_out;
  float* fbuf;     // [mp] F exchange
  float* gbuf;     // [mp] G exchange
  double* rs;      // [W] residual partials
  uint32_t* ctl;   // barrier counter, abort flag, ...
  double* dstats;
};

// LSE2 over a padded LDS row `row` (length mp) plus `vec`, by a group of kRedLPR lanes.
__device__ __forceinline__ float group_lse2(const float* __restrict__ row,
                                            const float* __restrict__ vec, int mp, int gl) {
  float M = kNegBig;
  for (int q = gl * 4; q < mp; q += kRedChunk) {
    const float4 l = *reinterpret_cast<const float4*>(row + q);
    const float4 v = *reinterpret_cast<const float4*>(vec + q);
    M = fmaxf(M, fmaxf(fmaxf(l.x + v.x, l.y + v.y), fmaxf(l.z + v.z, l.w + v.w)));
  }
  M = group_max(M, kRedLPR);
  float S = 0.0f;
  for (int q = gl * 4; q < mp; q += kRedChunk) {
    const float4 l = *reinterpret_cast<const float4*>(row + q);
    const float4 v = *reinterpret_cast<const float4*>(vec + q);
    S += exp2_fast(l.x + v.x - M) + exp2_fast(l.y + v.y - M) + exp2_fast(l.z + v.z - M) +
         exp2_fast(l.w + v.w - M);
  }
  S = group_sum(S, kRedLPR);
  return M + log2_fast(S);
}

__global__ void __launch_bounds__(kRedThreads) reduced_solver_kernel(RedParams p) {
  extern __shared__ float4 lds4[];
  float* lds = reinterpret_cast<float*>(lds4);
  const int R = p.R, mp = p.mp, m = p.m;
  float* Ls = lds;                      // [R][mp] row slab
  float* LTs = Ls + (size_t)R * mp;     // [R][mp] column slab (transposed)
  float* Vs = LTs + (size_t)R * mp;     // [mp] exchanged potential
  float* la2 = Vs + mp;                 // [R] log2 alpha (my rows)
  float* lb2 = la2 + R;                 // [R] log2 beta (my columns)
  float* Fcur = lb2 + R;                // [R]
  float* Fprev = Fcur + R;              // [R]
  float* Gcur = Fprev + R;              // [R]
  double* red = reinterpret_cast<double*>(Gcur + R + (R & 1));  // [8] reduction scratch
  __shared__ int s_flag;
  __shared__ int s_stop;

  const int w = blockIdx.x;
  const int r0 = w * R;
  const int nr = max(0, min(R, m - r0));  // rows (= columns) this workgroup owns
  const int tid = threadIdx.x;

  // ---- load the slabs (once) ------------------------------------------------------------
  for (int e = tid; e < R * mp; e += blockDim.x) {
    const int rl = e / mp, j = e - rl * mp;
    const bool ok = rl < nr && j < m;
    Ls[e] = ok ? p.logK[(int64_t)(r0 + rl) * m + j] * kLog2e : -INFINITY;
  }
  for (int e = tid; e < R * mp; e += blockDim.x) {
    const int i = e / R, cl = e - i * R;  // consecutive threads read consecutive columns
    if (i < mp) {
      const bool ok = cl < nr && i < m;
      LTs[(size_t)cl * mp + i] = ok ? p.logK[(int64_t)i * m + r0 + cl] * kLog2e : -INFINITY;
    }
  }
  for (int rl = tid; rl < R; rl += blockDim.x) {
    const bool ok = rl < nr;
    la2[rl] = ok ? log2f(p.alpha[r0 + rl]) : 0.0f;
    lb2[rl] = ok ? log2f(p.beta[r0 + rl]) : 0.0f;
    Gcur[rl] = ok && p.warm ? p.g_out[r0 + rl] * p.s2 : 0.0f;
    Fcur[rl] = 0.0f;
    Fprev[rl] = 0.0f;
  }
  for (int j = tid; j < mp; j += blockDim.x)
    Vs[j] = (j < m && p.warm) ? p.g_out[j] * p.s2 : 0.0f;
  __syncthreads();

  const int lane = tid & (kWave - 1);
  const int gl = lane % kRedLPR;                     // lane within its group
  const int grp = tid / kRedLPR;                     // group index in the block
  const int ngrp = blockDim.x / kRedLPR;
  uint32_t bar = 0;
  int iters_done = 0, converged = 0, flags = 0;
  double err2 = 0.0;

  for (int t = 1;; ++t) {
    // ---- row update: F^t from G^{t-1} (in Vs) -------------------------------------------
    double rpart = 0.0;
    for (int rl = grp; rl < nr; rl += ngrp) {
      const float lse = group_lse2(Ls + (size_t)rl * mp, Vs, mp, gl);
      const float Fn = la2[rl] - lse;
      if (gl == 0) {
        if (t >= 2) {
          const float rr = p.alpha[r0 + rl] * expm1f((Fcur[rl] - Fn) * kLn2);
          rpart += (double)rr * (double)rr;
        }
        Fprev[rl] = Fcur[rl];
        Fcur[rl] = Fn;
        p.fbuf[r0 + rl] = Fn;
      }
    }
    const double rtot = block_sum_d(rpart, red);
    if (tid == 0) p.rs[w] = rtot;
    if (!grid_barrier(p.ctl, (uint32_t)p.W * (++bar), &s_flag)) { flags |= 2; break; }

    // ---- stop test on the state after iteration t-1 --------------------------------------
    if (tid == 0) {
      int stop = 0;
      if (t >= 2) {
        double s = 0.0;
        for (int v = 0; v < p.W; ++v)
          s += __hip_atomic_load(&p.rs[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        err2 = s;
        const bool fin = s == s && s < 1.0e300;
        converged = fin && s <= p.tol2;
        // tol = 0 asks for exactly max_iter iterations, even if the residual underflows to 0
        stop = (converged && p.tol2 > 0.0) || !fin || (t - 1) >= p.max_iter;
        if (!fin) flags |= 1;
      }
      s_stop = stop;
    }
    __syncthreads();
    if (s_stop) { iters_done = t - 1; break; }

    // ---- column update: G^t from F^t -----------------------------------------------------
    for (int j = tid; j < mp; j += blockDim.x)
      Vs[j] = j < m ? __hip_atomic_load(&p.fbuf[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                    : 0.0f;
    __syncthreads();
    for (int cl = grp; cl < nr; cl += ngrp) {
      const float lse = group_lse2(LTs + (size_t)cl * mp, Vs, mp, gl);
      const float Gn = lb2[cl] - lse;
      if (gl == 0) {
        Gcur[cl] = Gn;
        p.gbuf[r0 + cl] = Gn;
      }
    }
    if (!grid_barrier(p.ctl, (uint32_t)p.W * (++bar), &s_flag)) { flags |= 2; break; }
    for (int j = tid; j < mp; j += blockDim.x)
      Vs[j] = j < m ? __hip_atomic_load(&p.gbuf[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                    : 0.0f;
    __syncthreads();
  }

  // ---- outputs: the state after iteration iters_done ------------------------------------
  __syncthreads();
  for (int rl = tid; rl < nr; rl += blockDim.x) {
    p.f_out[r0 + rl] = Fprev[rl] * p.to_nat;
    p.g_out[r0 + rl] = Gcur[rl] * p.to_nat;
  }
  if (w == 0 && tid == 0) {
    p.dstats[0] = (double)iters_done;
    p.dstats[1] = (double)converged;
    p.dstats[4] = sqrt((double)p.K * err2);
    p.dstats[5] = (double)flags;
  } else if (tid == 0 && flags) {
    p.dstats[5] = (double)flags;
  }
}

// ---- float64 marginal check -------------------------------------------------------------
// Blocks [0, nrb): four rows each (one wave per row); blocks [nrb, nrb + ncb): 64 columns
// each (lane = column, four row phases).  The last block to finish sums the partials.
__global__ void __launch_bounds__(256)
    reduced_check_kernel(int m, int K, double eps, const float* __restrict__ logK,
                         const float* __restrict__ f, const float* __restrict__ g,
                         const float* __restrict__ alpha, const float* __restrict__ beta,
                         double* __restrict__ part, uint32_t* __restrict__ counter,
                         double* __restrict__ dstats, int nrb, int ncb) {
  __shared__ double red[8];
  __shared__ double colacc[256];
  __shared__ int s_last;
  const double ie = 1.0 / eps;
  double r2 = 0.0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if ((int)blockIdx.x < nrb) {
    const int i = blockIdx.x * 4 + wv;
    if (i < m) {
      const double fi = f[i];
      double s = 0.0;
      for (int j = lane; j < m; j += 64)
        s += exp((double)logK[(int64_t)i * m + j] + (fi + (double)g[j]) * ie);
      s = wave_sum_d(s);
      const double d = s - (double)alpha[i];
      r2 = lane == 0 ? d * d : 0.0;
    }
  } else {
    const int j = (blockIdx.x - nrb) * 64 + lane;
    double s = 0.0;
    if (j < m) {
      const double gj = g[j];
      for (int i = wv; i < m; i += 4)
        s += exp((double)logK[(int64_t)i * m + j] + ((double)f[i] + gj) * ie);
    }
    colacc[threadIdx.x] = s;
    __syncthreads();
    if (wv == 0 && j < m) {
      const double c = colacc[lane] + colacc[lane + 64] + colacc[lane + 128] + colacc[lane + 192];
      const double d = c - (double)beta[j];
      r2 = d * d;
    }
  }
  const double tot = block_sum_d(r2, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = tot;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint32_t prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    s_last = prev == gridDim.x - 1;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  if (s_last && threadIdx.x == 0) {
    double er = 0.0, ec = 0.0;
    for (int b = 0; b < nrb; ++b) er += __hip_atomic_load(&part[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int b = nrb; b < nrb + ncb; ++b) ec += __hip_atomic_load(&part[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    dstats[2] = sqrt((double)K * er);
    dstats[3] = sqrt((double)K * ec);
    *counter = 0u;
  }
}

// ---- host side -------------------------------------------------------------------------

static int device_cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return cus;
}

static size_t reduced_lds_bytes(int R, int mp) {
  return sizeof(float) * ((size_t)2 * R * mp + mp + 5 * (size_t)R + 2) + 8 * sizeof(double) + 16;
}

bool plan_reduced(int m, int hint, ReducedPlan* plan) {
  const int cus = device_cu_count();
  if (cus <= 0) return false;
  const int mp = (m + kRedChunk - 1) / kRedChunk * kRedChunk;
  int W = hint;
  if (W <= 0) {
    // about 16 rows per workgroup, at most one workgroup per CU
    W = (m + 15) / 16;
    if (W < 1) W = 1;
    if (W > cus) W = cus;
  }
  if (W > m) W = m;
  int R = (m + W - 1) / W;
  W = (m + R - 1) / R;  // no empty workgroups
  size_t lds = reduced_lds_bytes(R, mp);
  while (lds > (size_t)kMaxLds && W < cus && W < m) {
    ++W;
    R = (m + W - 1) / W;
    W = (m + R - 1) / R;
    lds = reduced_lds_bytes(R, mp);
  }
  if (lds > (size_t)kMaxLds) return false;
  // co-residency: the cooperative launch needs all W workgroups resident at once
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute((const void*)reduced_solver_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds) != hipSuccess)
      return false;
    attr_set = true;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reduced_solver_kernel, kRedThreads,
                                                   lds) != hipSuccess)
    return false;
  if (per_cu * cus < W) return false;
  plan->W = W;
  plan->R = R;
  plan->threads = kRedThreads;
  plan->lds = lds;
  return true;
}

// workspace: ctl[64] words | fbuf[mp] | gbuf[mp] | rs[W] doubles | check partials
static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

size_t reduced_ws_bytes(int m, const ReducedPlan& p) {
  const int mp = (m + kRedChunk - 1) / kRedChunk * kRedChunk;
  const int nchk = (m + 3) / 4 + (m + 63) / 64;
  return align256(256) + 2 * align256(sizeof(float) * mp) + align256(sizeof(double) * p.W) +
         align256(sizeof(double) * nchk);
}

hipError_t launch_sinkhorn_reduced(int m, int K, double eps, const float* logK,
                                   const float* alpha, const float* beta, float* f, float* g,
                                   double tol, int max_iter, int warm, double* dstats,
                                   void* ws, const ReducedPlan& pl, hipStream_t s) {
  const int mp = (m + kRedChunk - 1) / kRedChunk * kRedChunk;
  char* base = static_cast<char*>(ws);
  uint32_t* ctl = reinterpret_cast<uint32_t*>(base);
  size_t off = align256(256);
  float* fbuf = reinterpret_cast<float*>(base + off); off += align256(sizeof(float) * mp);
  float* gbuf = reinterpret_cast<float*>(base + off); off += align256(sizeof(float) * mp);
  double* rs = reinterpret_cast<double*>(base + off); off += align256(sizeof(double) * pl.W);
  double* part = reinterpret_cast<double*>(base + off);

  hipError_t e = launch_zero_words(ctl, 64, s);
  if (e != hipSuccess) return e;

  RedParams p;
  p.m = m; p.mp = mp; p.K = K; p.W = pl.W; p.R = pl.R; p.max_iter = max_iter; p.warm = warm;
  p.s2 = (float)(kLog2eD / eps);
  p.to_nat = (float)(eps * kLn2D);
  p.tol2 = tol * tol / (double)K;
  p.logK = logK; p.alpha = alpha; p.beta = beta; p.f_out = f; p.g_out = g;
  p.fbuf = fbuf; p.gbuf = gbuf; p.rs = rs; p.ctl = ctl; p.dstats = dstats;
  void* args[] = {&p};
  e = hipLaunchCooperativeKernel((const void*)reduced_solver_kernel, dim3(pl.W),
                                 dim3(pl.threads), args, (unsigned)pl.lds, s);
  if (e != hipSuccess) return e;

  const int nrb = (m + 3) / 4, ncb = (m + 63) / 64;
  hipLaunchKernelGGL(reduced_check_kernel, dim3(nrb + ncb), dim3(256), 0, s, m, K, eps, logK,
                     f, g, alpha, beta, part, ctl + 8, dstats, nrb, ncb);
  return hipGetLastError();
}

}  // namespace csot
