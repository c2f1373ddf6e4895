// Plain full-size log-domain Sinkhorn on the n x n problem (the baseline the paper compares
// against: Alg. 3, stage 2, i.e. Cuturi's iteration), one persistent cooperative launch.
//
//   row    : F_I = log2 a_I - LSE2_J(G_J - C_IJ log2(e)/eps)
//   column : G_J = log2 b_J - LSE2_I(F_I - C_IJ log2(e)/eps)
//
// Workgroup w owns rows and columns [w R, w R + R).  In a row phase every workgroup streams
// the whole other side -- {coordinates, potential} packed as float4 -- through LDS in chunks
// of kNC points (double-buffered, next chunk prefetched into registers), and every lane
// evaluates costs on the fly for RT rows at a time (register blocking), keeping a running
// (max, sum) per row that is rescaled once per 4 columns.  Dense costs (dim = 0) are streamed
// from HBM instead: C for row phases, a transposed copy for column phases.  Phases are
// separated by device-wide barriers; the convergence test is the one of the reduced solver.
#include "common.hpp"
#include "launch.hpp"

namespace csot {

constexpr int kFullThreads = 256;  // 4 waves
constexpr int kNC = 1024;          // points per LDS chunk (16 KiB of float4)
constexpr int kPF = kNC / kFullThreads;

struct FullParams {
  int n, np, W, R, max_iter, warm;
  float s2, to_nat;
  double tol2;
  const float* x;
  const float* y;
  const float* C;
  int64_t ldc;
  const float* CT;   // dense transpose [n, np]
  const float* a;
  const float* b;
  float* f_out;
  float* g_out;
  float4* xf;        // [np] {x_I, F_I}
  float4* yg;        // [np] {y_J, G_J}
  double* rs;        // [W]
  uint32_t* ctl;
  double* dstats;
};

template <int DIM>
__device__ __forceinline__ float4 pack_point(const float* __restrict__ p, int I, float pot) {
  float4 v;
  v.x = p[(int64_t)I * DIM + 0];
  v.y = p[(int64_t)I * DIM + 1];
  v.z = DIM == 3 ? p[(int64_t)I * DIM + 2] : 0.0f;
  v.w = pot;
  return v;
}

// One phase: for the RT own rows of this wave, LSE2 over all other points.
// own: coordinates of the own side; other: packed other side (potential in .w).
template <int DIM, int RT>
__device__ __forceinline__ void full_phase(const FullParams& p, int r0,
                                           const float* __restrict__ own,
                                           const float* __restrict__ dense, int64_t ldd,
                                           const float4* __restrict__ other,
                                           float4* __restrict__ buf, float* __restrict__ lse) {
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  const int rbase = r0 + wv * RT;
  float xr[RT][3];
  float M[RT], S[RT];
  const float* drow[RT];
#pragma unroll
  for (int q = 0; q < RT; ++q) {
    const int I = min(rbase + q, p.n - 1);
    if constexpr (DIM > 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) xr[q][d] = d < DIM ? own[(int64_t)I * DIM + d] : 0.0f;
    }
    drow[q] = DIM == 0 ? dense + (int64_t)I * ldd : nullptr;
    M[q] = kNegBig;
    S[q] = 0.0f;
  }
  const int nchunks = p.np / kNC;
  float4 pre[kPF];
#pragma unroll
  for (int u = 0; u < kPF; ++u) pre[u] = other[tid + u * kFullThreads];
  for (int c = 0; c < nchunks; ++c) {
    float4* cur = buf + (c & 1) * kNC;
#pragma unroll
    for (int u = 0; u < kPF; ++u) cur[tid + u * kFullThreads] = pre[u];
    __syncthreads();
    if (c + 1 < nchunks) {
#pragma unroll
      for (int u = 0; u < kPF; ++u) pre[u] = other[(c + 1) * kNC + tid + u * kFullThreads];
    }
    for (int u = 0; u < kNC / kWave; u += 4) {
      float4 o[4];
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) o[cc] = cur[lane + kWave * (u + cc)];
#pragma unroll
      for (int q = 0; q < RT; ++q) {
        float t[4];
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          float cst;
          if constexpr (DIM == 0) {
            const int J = c * kNC + lane + kWave * (u + cc);
            cst = J < p.n ? drow[q][J] : 0.0f;
          } else {
            const float dx = xr[q][0] - o[cc].x;
            const float dy = xr[q][1] - o[cc].y;
            cst = dx * dx;
            cst = fmaf(dy, dy, cst);
            if constexpr (DIM == 3) {
              const float dz = xr[q][2] - o[cc].z;
              cst = fmaf(dz, dz, cst);
            }
          }
          t[cc] = fmaf(-cst, p.s2, o[cc].w);
        }
        const float tm = fmaxf(fmaxf(t[0], t[1]), fmaxf(t[2], t[3]));
        const float Mn = fmaxf(M[q], tm);
        S[q] = S[q] * exp2_fast(M[q] - Mn) + exp2_fast(t[0] - Mn) + exp2_fast(t[1] - Mn) +
               exp2_fast(t[2] - Mn) + exp2_fast(t[3] - Mn);
        M[q] = Mn;
      }
    }
  }
  // merge the 64 lanes' partials of each row
#pragma unroll
  for (int q = 0; q < RT; ++q) {
    float m_ = M[q], s_ = S[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const float m2 = __shfl_xor(m_, o, kWave);
      const float s2 = __shfl_xor(s_, o, kWave);
      lse_merge(m_, s_, m2, s2);
    }
    if (lane == 0) lse[wv * RT + q] = m_ + log2_fast(s_);
  }
  __syncthreads();
}

template <int DIM, int RT>
__global__ void __launch_bounds__(kFullThreads) full_solver_kernel(FullParams p) {
  __shared__ float4 buf[2 * kNC];
  __shared__ float lse[4 * RT];
  __shared__ float Fcur[4 * RT], Fprev[4 * RT], Gcur[4 * RT], la2[4 * RT], lb2[4 * RT];
  __shared__ double red[8];
  __shared__ int s_flag, s_stop;
  const int w = blockIdx.x, tid = threadIdx.x;
  const int R = p.R;  // == 4 * RT
  const int r0 = w * R;
  const int nr = max(0, min(R, p.n - r0));

  // ---- setup: publish own rows / columns, pad the exchange arrays -----------------------
  for (int rl = tid; rl < R; rl += blockDim.x) {
    const bool ok = rl < nr;
    const int I = r0 + rl;
    la2[rl] = ok ? log2f(p.a[I]) : 0.0f;
    lb2[rl] = ok ? log2f(p.b[I]) : 0.0f;
    Fcur[rl] = 0.0f;
    Fprev[rl] = 0.0f;
    const float G0 = ok && p.warm ? p.g_out[I] * p.s2 : 0.0f;
    Gcur[rl] = G0;
    if (ok) {
      if constexpr (DIM > 0) {
        p.xf[I] = pack_point<DIM>(p.x, I, 0.0f);
        p.yg[I] = pack_point<DIM>(p.y, I, G0);
      } else {
        p.xf[I] = make_float4(0.f, 0.f, 0.f, 0.f);
        p.yg[I] = make_float4(0.f, 0.f, 0.f, G0);
      }
    }
  }
  if (w == 0) {
    for (int I = p.n + tid; I < p.np; I += blockDim.x) {
      p.xf[I] = make_float4(0.f, 0.f, 0.f, -INFINITY);
      p.yg[I] = make_float4(0.f, 0.f, 0.f, -INFINITY);
    }
  }
  uint32_t bar = 0;
  int iters_done = 0, converged = 0, flags = 0;
  double err2 = 0.0;
  if (!grid_barrier(p.ctl, (uint32_t)p.W * (++bar), &s_flag)) flags |= 2;

  for (int t = 1; !(flags & 2); ++t) {
    // ---- row phase ----------------------------------------------------------------------
    full_phase<DIM, RT>(p, r0, p.x, p.C, p.ldc, p.yg, buf, lse);
    double rpart = 0.0;
    for (int rl = tid; rl < nr; rl += blockDim.x) {
      const int I = r0 + rl;
      const float Fn = la2[rl] - lse[rl];
      if (t >= 2) {
        const float rr = p.a[I] * expm1f((Fcur[rl] - Fn) * kLn2);
        rpart += (double)rr * (double)rr;
      }
      Fprev[rl] = Fcur[rl];
      Fcur[rl] = Fn;
      float4 v = DIM > 0 ? pack_point<(DIM > 0 ? DIM : 2)>(p.x, I, Fn) : make_float4(0.f, 0.f, 0.f, Fn);
      p.xf[I] = v;
    }
    const double rtot = block_sum_d(rpart, red);
    if (tid == 0) p.rs[w] = rtot;
    if (!grid_barrier(p.ctl, (uint32_t)p.W * (++bar), &s_flag)) { flags |= 2; break; }
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

    // ---- column phase -------------------------------------------------------------------
    full_phase<DIM, RT>(p, r0, p.y, p.CT, p.np, p.xf, buf, lse);
    for (int cl = tid; cl < nr; cl += blockDim.x) {
      const int J = r0 + cl;
      const float Gn = lb2[cl] - lse[cl];
      Gcur[cl] = Gn;
      float4 v = DIM > 0 ? pack_point<(DIM > 0 ? DIM : 2)>(p.y, J, Gn) : make_float4(0.f, 0.f, 0.f, Gn);
      p.yg[J] = v;
    }
    if (!grid_barrier(p.ctl, (uint32_t)p.W * (++bar), &s_flag)) { flags |= 2; break; }
  }

  __syncthreads();
  for (int rl = tid; rl < nr; rl += blockDim.x) {
    p.f_out[r0 + rl] = Fprev[rl] * p.to_nat;
    p.g_out[r0 + rl] = Gcur[rl] * p.to_nat;
  }
  if (w == 0 && tid == 0) {
    p.dstats[0] = (double)iters_done;
    p.dstats[1] = (double)converged;
    p.dstats[4] = sqrt(err2);
    p.dstats[5] = (double)flags;
  } else if (tid == 0 && flags) {
    p.dstats[5] = (double)flags;
  }
}

// ---- dense transpose (dim = 0): CT[j, i] = C[i, j], CT [n, np] --------------------------
__global__ void transpose_kernel(const float* __restrict__ C, int64_t ldc, float* __restrict__ CT,
                                 int64_t ldt, int n) {
  __shared__ float tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int i = by + k, j = bx + tx;
    tile[k][tx] = (i < n && j < n) ? C[(int64_t)i * ldc + j] : 0.0f;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int j = bx + k, i = by + tx;
    if (i < n && j < n) CT[(int64_t)j * ldt + i] = tile[tx][k];
  }
}

// ---- float64 marginal check of the full plan ------------------------------------------
// Tile of 32 rows x 64 columns per block; row and column partial sums go to double
// accumulators with atomics; the last block forms the two norms.
template <int DIM>
__global__ void __launch_bounds__(256)
    full_check_kernel(FullParams p, double eps, double* __restrict__ rowsum,
                      double* __restrict__ colsum, uint32_t* __restrict__ counter, int ntiles) {
  __shared__ double cpart[4][64];
  __shared__ double red[8];
  __shared__ int s_last;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int J = blockIdx.x * 64 + lane;
  const int I0 = blockIdx.y * 32;
  const double ie = 1.0 / eps;
  double csum = 0.0;
  const double gJ = J < p.n ? (double)p.g_out[J] : 0.0;
  for (int q = 0; q < 8; ++q) {
    const int I = I0 + wv + 4 * q;
    double v = 0.0;
    if (I < p.n && J < p.n) {
      double c;
      if constexpr (DIM == 0) {
        c = (double)p.C[(int64_t)I * p.ldc + J];
      } else {
        c = 0.0;
        for (int d = 0; d < DIM; ++d) {
          const double df = (double)p.x[(int64_t)I * DIM + d] - (double)p.y[(int64_t)J * DIM + d];
          c += df * df;
        }
      }
      v = exp(((double)p.f_out[I] + gJ - c) * ie);
    }
    csum += v;
    const double rs = wave_sum_d(v);
    if (lane == 0 && I < p.n) atomicAdd(&rowsum[I], rs);
  }
  cpart[wv][lane] = csum;
  __syncthreads();
  if (wv == 0 && J < p.n)
    atomicAdd(&colsum[J], cpart[0][lane] + cpart[1][lane] + cpart[2][lane] + cpart[3][lane]);
  // last block: norms
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_last = prev == (uint32_t)ntiles - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  double er = 0.0, ec = 0.0;
  for (int I = threadIdx.x; I < p.n; I += blockDim.x) {
    const double dr = __hip_atomic_load(&rowsum[I], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - (double)p.a[I];
    const double dc = __hip_atomic_load(&colsum[I], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - (double)p.b[I];
    er += dr * dr;
    ec += dc * dc;
  }
  er = block_sum_d(er, red);
  ec = block_sum_d(ec, red);
  if (threadIdx.x == 0) {
    p.dstats[2] = sqrt(er);
    p.dstats[3] = sqrt(ec);
  }
}

__global__ void zero_doubles_kernel(double* p, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// ---- host side -------------------------------------------------------------------------
static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

static int cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return cus;
}

template <int DIM, int RT>
static const void* full_kernel_ptr() { return (const void*)full_solver_kernel<DIM, RT>; }

static const void* pick_full_kernel(int dim, int RT) {
#define CSOT_FK(D)                                    \
  switch (RT) {                                       \
    case 1: return full_kernel_ptr<D, 1>();           \
    case 2: return full_kernel_ptr<D, 2>();           \
    case 4: return full_kernel_ptr<D, 4>();           \
    case 8: return full_kernel_ptr<D, 8>();           \
    default: return nullptr;                          \
  }
  switch (dim) {
    case 0: CSOT_FK(0)
    case 2: CSOT_FK(2)
    case 3: CSOT_FK(3)
    default: return nullptr;
  }
#undef CSOT_FK
}

bool plan_full(const Geom& g, int hint, FullPlan* plan) {
  const int cus = cu_count();
  if (cus <= 0) return false;
  int RT = 1;
  if (hint > 0) {
    // rows per wave from the requested workgroup count
    const int rows = (g.n + hint - 1) / hint;
    RT = rows <= 4 ? 1 : rows <= 8 ? 2 : rows <= 16 ? 4 : 8;
  } else {
    for (int cand : {8, 4, 2, 1}) {
      if ((g.n + 4 * cand - 1) / (4 * cand) >= cus) { RT = cand; break; }
    }
  }
  const int R = 4 * RT;
  const int W = (g.n + R - 1) / R;
  const void* k = pick_full_kernel(g.dim, RT);
  if (!k) return false;
  int per_cu = 0;
  hipError_t e = hipSuccess;
  switch (g.dim) {  // occupancy query needs the typed kernel
#define CSOT_OCC(D)                                                                        \
  e = RT == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, full_solver_kernel<D, 1>, kFullThreads, 0) \
    : RT == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, full_solver_kernel<D, 2>, kFullThreads, 0) \
    : RT == 4 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, full_solver_kernel<D, 4>, kFullThreads, 0) \
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, full_solver_kernel<D, 8>, kFullThreads, 0);
    case 0: CSOT_OCC(0) break;
    case 2: CSOT_OCC(2) break;
    case 3: CSOT_OCC(3) break;
    default: return false;
#undef CSOT_OCC
  }
  if (e != hipSuccess || per_cu * cus < W) return false;
  plan->W = W;
  plan->R = R;
  plan->threads = kFullThreads;
  plan->lds = 0;
  return true;
}

// workspace: ctl | xf[np] | yg[np] | rs[W] | rowsum[n] | colsum[n] | CT[n*np] (dense)
size_t full_ws_bytes(const Geom& g, const FullPlan& pl) {
  const size_t np = (size_t)((g.n + kNC - 1) / kNC * kNC);
  size_t b = align256(256) + 2 * align256(sizeof(float4) * np) + align256(sizeof(double) * pl.W) +
             2 * align256(sizeof(double) * g.n);
  if (g.dim == 0) b += align256(sizeof(float) * (size_t)g.n * np);
  return b;
}

hipError_t launch_sinkhorn_full(const Geom& g, float* f, float* gpot, double tol, int max_iter,
                                int warm, double* dstats, void* ws, const FullPlan& pl,
                                hipStream_t s) {
  const int np = (g.n + kNC - 1) / kNC * kNC;
  char* base = static_cast<char*>(ws);
  uint32_t* ctl = reinterpret_cast<uint32_t*>(base);
  size_t off = align256(256);
  float4* xf = reinterpret_cast<float4*>(base + off); off += align256(sizeof(float4) * np);
  float4* yg = reinterpret_cast<float4*>(base + off); off += align256(sizeof(float4) * np);
  double* rs = reinterpret_cast<double*>(base + off); off += align256(sizeof(double) * pl.W);
  double* rowsum = reinterpret_cast<double*>(base + off); off += align256(sizeof(double) * g.n);
  double* colsum = reinterpret_cast<double*>(base + off); off += align256(sizeof(double) * g.n);
  float* CT = reinterpret_cast<float*>(base + off);

  hipError_t e = launch_zero_words(ctl, 64, s);
  if (e != hipSuccess) return e;
  if (g.dim == 0) {
    hipLaunchKernelGGL(transpose_kernel, dim3((g.n + 31) / 32, (g.n + 31) / 32), dim3(256), 0, s,
                       g.C, g.ldc, CT, (int64_t)np, g.n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  FullParams p;
  p.n = g.n; p.np = np; p.W = pl.W; p.R = pl.R; p.max_iter = max_iter; p.warm = warm;
  p.s2 = (float)(kLog2eD / g.eps);
  p.to_nat = (float)(g.eps * kLn2D);
  p.tol2 = tol * tol;
  p.x = g.x; p.y = g.y; p.C = g.C; p.ldc = g.ldc; p.CT = CT; p.a = g.a; p.b = g.b;
  p.f_out = f; p.g_out = gpot; p.xf = xf; p.yg = yg; p.rs = rs; p.ctl = ctl; p.dstats = dstats;
  void* args[] = {&p};
  const void* k = pick_full_kernel(g.dim, pl.R / 4);
  if (!k) return hipErrorInvalidValue;
  e = hipLaunchCooperativeKernel(k, dim3(pl.W), dim3(pl.threads), args, 0, s);
  if (e != hipSuccess) return e;

  // float64 check
  hipLaunchKernelGGL(zero_doubles_kernel, dim3(64), dim3(256), 0, s, rowsum,
                     (int64_t)(align256(sizeof(double) * g.n) / sizeof(double)) * 2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const dim3 grid((g.n + 63) / 64, (g.n + 31) / 32);
  const int ntiles = grid.x * grid.y;
  switch (g.dim) {
    case 0: hipLaunchKernelGGL(full_check_kernel<0>, grid, dim3(256), 0, s, p, g.eps, rowsum, colsum, ctl + 8, ntiles); break;
    case 2: hipLaunchKernelGGL(full_check_kernel<2>, grid, dim3(256), 0, s, p, g.eps, rowsum, colsum, ctl + 8, ntiles); break;
    case 3: hipLaunchKernelGGL(full_check_kernel<3>, grid, dim3(256), 0, s, p, g.eps, rowsum, colsum, ctl + 8, ntiles); break;
  }
  return hipGetLastError();
}

}  // namespace csot
