// Plain full-size log-domain Sinkhorn on the n x n problem (the baseline the paper compares
// against: Alg. 3, stage 2, i.e. Cuturi's iteration), one persistent launch.
//
//   row    : F_I = log2 a_I - LSE2_J(G_J - C_IJ log2(e)/eps)
//   column : G_J = log2 b_J - LSE2_I(F_I - C_IJ log2(e)/eps)
//
// Workgroup w owns rows and columns [w R, w R + R).  It runs 16 waves: RG row groups of RT
// rows (register blocking: one staged column feeds RT rows) times CQ column parts.  In a
// row phase the whole other side streams through LDS in chunks of kNC points -- static
// coordinates (packed once per solve) plus the current potential, read from epoch-tagged
// 64-bit slots and polled until they carry the current iteration -- double-buffered with the
// next chunk prefetched into registers.  Every lane evaluates costs on the fly from
// coordinates pre-scaled by sqrt(log2(e)/eps), so that an exponent is G_J - |x'_I - y'_J|^2;
// lanes, then column parts, are merged at the end.  Dense costs (dim = 0) are streamed from HBM instead: C for row
// phases, a transposed copy for column phases.  Exchange and stop test are those of the
// reduced solver (slots as their own ready flags, no counter barrier, no cache flushes).
#include "common.hpp"
#include "launch.hpp"

namespace csot {

constexpr int kFullThreads = 1024;  // 16 waves
constexpr int kFullWaves = kFullThreads / kWave;
constexpr int kNC = 2048;           // points per LDS chunk (two per thread)
constexpr int kPF = kNC / kFullThreads;

struct FullParams {
  int n, np, W, R, P, max_iter;  // P row blocks of R rows per workgroup
  float s2, to_nat;
  double tol2;
  const float4* xc;  // [np] packed x coordinates
  const float4* yc;  // [np] packed y coordinates
  const float* C;
  int64_t ldc;
  const float* CT;   // dense transpose [n, np]
  const float* a;
  const float* b;
  float* f_out;
  float* g_out;
  uint64_t* fx;      // [np] F slots (epoch t = row phase of iteration t)
  uint64_t* gx;      // [np] G slots (epoch 0 = initial potential)
  uint64_t* rsx;     // [W] residual partials
  uint32_t* ctl;     // [0] abort flag
  double* dstats;
};

// Smallest shifted row sum the shifted mode accepts: every dropped term is below 2^-126, so
// with n < 2^24 the lost mass stays below 2^-42 of the accepted sum.
constexpr float kMinShiftedSum = 0x1p-60f;

// One phase for this workgroup's rows: LSE2 over all other points of (pot_J - C_IJ s2).
// lse[rl] receives the result for local row rl.  Returns kPhaseOk, kPhaseAbort, or (shifted
// mode only) kPhaseRedo when a row's shifted sum fell outside [2^-60, inf).
//
// Exact mode keeps a running (max, sum) per row, rescaled once per 4 columns.  Shifted mode
// needs no maximum: it sums 2^(pot_J + sig - C_IJ s2) with one shift sig per workgroup, the
// largest previous potential sh_I of its rows.  With sh_I in place of sig the sum would be the
// previous plan's row sum (every term of a row is at most the other side's marginal entry
// after that side's last update), at most 1; the common shift scales it by 2^(sig - sh_I) >= 1,
// so it cannot underflow where the row's own shift would not, and overflows only when the
// workgroup's previous potentials spread over more than ~127 (base 2).  Either case (a sum
// outside [2^-60, inf)) makes the caller redo the phase in exact mode.  The shift is added to
// the staged potentials, so an entry costs 2 sub, 2 fma, 1 exp and 1 add (dim 2).
constexpr int kPhaseOk = 0, kPhaseAbort = 1, kPhaseRedo = 2;

// The used coordinates of a packed point, loaded at their own width: a full float4 load would
// also write the register that the staged potential later takes, and a register written by a
// load still in flight cannot be reused before the load completes.
template <int DIM>
__device__ __forceinline__ float4 load_coords(const float4* __restrict__ c) {
  if constexpr (DIM == 0) {
    return make_float4(0.f, 0.f, 0.f, 0.f);
  } else {
    const float2 v = *reinterpret_cast<const float2*>(c);
    const float z = DIM == 3 ? reinterpret_cast<const float*>(c)[2] : 0.0f;
    return make_float4(v.x, v.y, z, 0.0f);
  }
}

// WIDE (shifted mode only): the workgroup's previous potentials spread too far for one common
// shift; each row group (the RT rows of a wave) then shifts by its own largest previous
// potential, added to the staged value once per column and wave (an add per RT entries).
template <int DIM, int RT, int CQ, bool EXACT, bool WIDE = false>
__device__ __forceinline__ int full_phase(const FullParams& p, int r0, const float4* __restrict__ ownc,
                                          const float* __restrict__ dense, int64_t ldd,
                                          const float4* __restrict__ othc, uint64_t* oslots,
                                          uint32_t epoch, const float* __restrict__ sh,
                                          float4* __restrict__ buf, float2* __restrict__ part,
                                          float* __restrict__ lse, int* s_bad, int* s_redo,
                                          uint64_t* xs, int nx, uint32_t xepoch,
                                          float* __restrict__ xdst) {
  constexpr int RG = kFullWaves / CQ;
  constexpr int U = kNC / kWave / CQ;  // 64-column steps per wave per chunk
  constexpr int TU = U < 4 ? U : 4;     // columns per lane between running-max rescales
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int rg = wv / CQ, cq = wv % CQ;
  float xr[RT][3];
  float M[RT], S[RT];
  const float* drow[RT];
#pragma unroll
  for (int q = 0; q < RT; ++q) {
    const int rl = rg * RT + q;
    const int I = min(r0 + rl, p.n - 1);
    if constexpr (DIM > 0) {
      const float4 c = ownc[I];
      xr[q][0] = c.x; xr[q][1] = c.y; xr[q][2] = c.z;
    }
    drow[q] = DIM == 0 ? dense + (int64_t)I * ldd : nullptr;
    M[q] = kNegBig;
    S[q] = 0.0f;
  }
  // the workgroup's common shift: its rows' largest previous potential (written before the
  // barrier that ended the previous update; R <= 64 rows, one per lane, and every wave gets
  // the bitwise-identical maximum)
  float sig = 0.0f, dsig = 0.0f;
  if constexpr (!EXACT) {
    static_assert(RG * RT <= kWave, "one row per lane");
    sig = wave_max_v(lane < RG * RT && r0 + lane < p.n ? sh[lane] : kNegBig);
    if constexpr (WIDE) {
      float gs = kNegBig;  // this row group's largest previous potential
#pragma unroll
      for (int q = 0; q < RT; ++q)
        if (r0 + rg * RT + q < p.n) gs = fmaxf(gs, sh[rg * RT + q]);
      dsig = gs - sig;  // <= 0
    }
  }
  if (tid == 0) *s_redo = 0;
  const int nchunks = p.np / kNC;
  bool ok = true;
  // prefetch chunk 0: coordinates and slots of points tid + k * kFullThreads; the nx extra
  // slots xs[] (another exchange, long published) are staged into xdst with the last chunk
  float4 pc[kPF];
  uint64_t ps[kPF];
  uint64_t xw = 0;
#pragma unroll
  for (int k = 0; k < kPF; ++k) {
    const int J = tid + k * kFullThreads;
    pc[k] = load_coords<DIM>(othc + J);
    ps[k] = J < p.n ? slot_load(oslots + J) : 0ull;
  }
  if (nchunks == 1 && tid < nx) xw = slot_load(xs + tid);
  for (int c = 0; c < nchunks; ++c) {
    float4* cur = buf + (c & 1) * kNC;
#pragma unroll
    for (int k = 0; k < kPF; ++k) {
      const int J = c * kNC + tid + k * kFullThreads;
      if (J < p.n) {
        if (ok) ok = slot_wait(oslots + J, ps[k], epoch, p.ctl);
        pc[k].w = slot_value(ps[k]) + sig;
      } else {
        pc[k].w = -INFINITY;
      }
      cur[tid + k * kFullThreads] = pc[k];
    }
    if (c == nchunks - 1 && tid < nx) {
      if (ok) ok = slot_wait(xs + tid, xw, xepoch, p.ctl);
      xdst[tid] = slot_value(xw);
    }
    if (!ok) *s_bad = 1;
    __syncthreads();
    if (*s_bad) return kPhaseAbort;
    if (c + 1 < nchunks) {
#pragma unroll
      for (int k = 0; k < kPF; ++k) {
        const int Jn = (c + 1) * kNC + tid + k * kFullThreads;
        pc[k] = load_coords<DIM>(othc + Jn);
        ps[k] = Jn < p.n ? slot_load(oslots + Jn) : 0ull;
      }
      if (c + 2 == nchunks && tid < nx) xw = slot_load(xs + tid);
    }
#pragma unroll 1
    for (int u = cq * U; u < (cq + 1) * U; u += TU) {
      float4 o[TU];
#pragma unroll
      for (int cc = 0; cc < TU; ++cc) {
        o[cc] = cur[lane + kWave * (u + cc)];
        if constexpr (WIDE) o[cc].w += dsig;
      }
#pragma unroll
      for (int q = 0; q < RT; ++q) {
        float t[TU];
#pragma unroll
        for (int cc = 0; cc < TU; ++cc) {
          if constexpr (DIM == 0) {
            const int Jc = c * kNC + lane + kWave * (u + cc);
            t[cc] = fmaf(-(Jc < p.n ? drow[q][Jc] : 0.0f), p.s2, o[cc].w);
          } else {
            // scaled coordinates: -C_IJ s2 = -|x'_I - y'_J|^2
            const float dx = xr[q][0] - o[cc].x;
            const float dy = xr[q][1] - o[cc].y;
            float e = fmaf(-dx, dx, o[cc].w);
            e = fmaf(-dy, dy, e);
            if constexpr (DIM == 3) {
              const float dz = xr[q][2] - o[cc].z;
              e = fmaf(-dz, dz, e);
            }
            t[cc] = e;
          }
        }
        if constexpr (EXACT) {
          float tm = t[0];
#pragma unroll
          for (int cc = 1; cc < TU; ++cc) tm = fmaxf(tm, t[cc]);
          const float Mn = fmaxf(M[q], tm);
          float acc = S[q] * exp2_fast(M[q] - Mn);
#pragma unroll
          for (int cc = 0; cc < TU; ++cc) acc += exp2_fast(t[cc] - Mn);
          S[q] = acc;
          M[q] = Mn;
        } else {
#pragma unroll
          for (int cc = 0; cc < TU; ++cc) S[q] += exp2_fast(t[cc]);
        }
      }
    }
  }
  // merge the 64 lanes of each row, then the CQ column parts
#pragma unroll
  for (int q = 0; q < RT; ++q) {
    float m_ = M[q], s_ = S[q];
    if constexpr (EXACT) {
      wave_lse_merge(m_, s_);
    } else {
      s_ = wave_sum_v(s_);
    }
    if (lane == 0) part[(rg * RT + q) * CQ + cq] = make_float2(m_, s_);
  }
  __syncthreads();
  for (int rl = tid; rl < RG * RT; rl += kFullThreads) {
    if constexpr (EXACT) {
      float m_ = kNegBig, s_ = 0.0f;
      for (int k = 0; k < CQ; ++k) {
        const float2 v = part[rl * CQ + k];
        lse_merge(m_, s_, v.x, v.y);
      }
      lse[rl] = m_ + log2_fast(s_);
    } else {
      float s_ = 0.0f;
      for (int k = 0; k < CQ; ++k) s_ += part[rl * CQ + k].y;
      float rs = sig;  // the shift this row's sums carry
      if constexpr (WIDE) {
        const int g0 = rl / RT * RT;
        rs = kNegBig;
        for (int q = 0; q < RT; ++q)
          if (r0 + g0 + q < p.n) rs = fmaxf(rs, sh[g0 + q]);
      }
      if (r0 + rl < p.n && !(s_ >= kMinShiftedSum && s_ < INFINITY)) *s_redo = 1;
      lse[rl] = log2_fast(s_) - rs;
    }
  }
  __syncthreads();
  return (!EXACT && *s_redo) ? kPhaseRedo : kPhaseOk;
}

// A phase in shifted mode, redone in exact mode when the shifted sums are out of range.
template <int DIM, int RT, int CQ>
__device__ __forceinline__ int full_phase_auto(bool exact, const FullParams& p, int r0,
                                               const float4* ownc, const float* dense,
                                               int64_t ldd, const float4* othc,
                                               uint64_t* oslots, uint32_t epoch,
                                               const float* sh, float4* buf, float2* part,
                                               float* lse, int* s_bad, int* s_redo,
                                               int* redo_count, uint64_t* xs = nullptr,
                                               int nx = 0, uint32_t xepoch = 0,
                                               float* xdst = nullptr) {
  if (!exact) {
    // spread of the rows' previous potentials: beyond ~100 (base 2) the common shift (the
    // largest of them) would scale the sums of the lowest rows towards float32 overflow, so
    // each row group shifts by its own largest
    constexpr int NR = (kFullWaves / CQ) * RT;
    const int lane = threadIdx.x & (kWave - 1);
    const bool in = lane < NR && r0 + lane < p.n;
    const float hi = wave_max_v(in ? sh[lane] : kNegBig);
    const float lo = -wave_max_v(in ? -sh[lane] : kNegBig);
    const int r = hi - lo > 100.0f
                      ? full_phase<DIM, RT, CQ, false, true>(p, r0, ownc, dense, ldd, othc,
                                                             oslots, epoch, sh, buf, part, lse,
                                                             s_bad, s_redo, xs, nx, xepoch, xdst)
                      : full_phase<DIM, RT, CQ, false>(p, r0, ownc, dense, ldd, othc, oslots,
                                                       epoch, sh, buf, part, lse, s_bad, s_redo,
                                                       xs, nx, xepoch, xdst);
    if (r != kPhaseRedo) return r;
    ++*redo_count;
    __syncthreads();  // every wave is done with the chunk buffers
  }
  return full_phase<DIM, RT, CQ, true>(p, r0, ownc, dense, ldd, othc, oslots, epoch, sh, buf,
                                       part, lse, s_bad, s_redo, xs, nx, xepoch, xdst);
}

constexpr int kMaxRowBlocks = 4;  // row blocks per workgroup (n up to 4 x 64 x workgroups)

template <int DIM, int RT, int CQ>
__global__ void __launch_bounds__(kFullThreads) full_solver_kernel(FullParams p) {
  constexpr int R = (kFullWaves / CQ) * RT;
  static_assert(R <= kWave, "a row block's rows are one per lane of wave 0");
  constexpr int RM = kMaxRowBlocks * R;
  __shared__ float4 buf[2 * kNC];
  __shared__ float2 part[R * CQ];
  __shared__ float lse[RM];
  __shared__ float Fcur[RM], Fprev[RM], Gcur[RM], Gprev[RM], la2[RM], lb2[RM], aa[RM];
  __shared__ float rsl[kFullThreads];  // residual partials of all workgroups (W <= 1024)
  __shared__ int s_bad, s_redo;
  const int w = blockIdx.x, tid = threadIdx.x;
  const int P = p.P;
  // workgroup w owns rows [w P R, (w + 1) P R): P blocks of R rows, each a pass over the
  // other side
  const int rbase = w * P * R;
  const int nr = max(0, min(P * R, p.n - rbase));
  const int nb = (nr + R - 1) / R;  // row blocks holding rows

  for (int rl = tid; rl < P * R; rl += blockDim.x) {
    const bool ok = rl < nr;
    const int I = rbase + rl;
    aa[rl] = ok ? p.a[I] : 0.0f;
    la2[rl] = ok ? log2f(p.a[I]) : 0.0f;
    lb2[rl] = ok ? log2f(p.b[I]) : 0.0f;
    Fcur[rl] = 0.0f;
    Fprev[rl] = 0.0f;
    Gcur[rl] = ok ? slot_value(slot_load(p.gx + I)) : 0.0f;  // initial G (epoch 0)
    Gprev[rl] = Gcur[rl];
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();
  int iters_done = 0, converged = 0, flags = 0, redos = 0;
  double err2 = 0.0;

  // Iteration t: row phase (F^t from G^{t-1}), then column phase (G^t from F^t).  The row
  // update also yields the residual of the state after iteration t-1; every workgroup
  // publishes its partial, and the column phase stages all of them into LDS with its last
  // chunk, when they have long been visible, so the stop test never holds up the exchange.
  // Every wave then sums the same partials in the same order and takes the same decision; a
  // stop at iteration t returns the state after t-1 (F^{t-1}, G^{t-1}) and discards the
  // column phase just done.
  for (uint32_t t = 1;; ++t) {
    // ---- row phase: F^t from G^{t-1} ----------------------------------------------------
    // F^1 has no previous F to shift by: exact mode; later rows shift by F^{t-1}
    int st = kPhaseOk;
    for (int b = 0; b < nb && st == kPhaseOk; ++b)
      st = full_phase_auto<DIM, RT, CQ>(t == 1, p, rbase + b * R, p.xc, p.C, p.ldc, p.yc, p.gx,
                                        t - 1, Fcur + b * R, buf, part, lse + b * R, &s_bad,
                                        &s_redo, &redos);
    if (st != kPhaseOk) {
      flags |= 2;
      break;
    }
    if (tid < kWave) {  // wave 0: one row per lane and block
      float rr2 = 0.0f;
      for (int rl = tid; rl < nr; rl += kWave) {
        const float Fn = la2[rl] - lse[rl];
        if (t >= 2) {
          const float rr = scaled_exp2m1(aa[rl], Fcur[rl] - Fn);
          rr2 = fmaf(rr, rr, rr2);
        }
        Fprev[rl] = Fcur[rl];
        Fcur[rl] = Fn;
        slot_publish(p.fx + rbase + rl, Fn, t);
      }
      rr2 = wave_sum_v(rr2);  // vector-unit reduction (DPP, lane swaps)
      if (tid == 0) slot_publish(p.rsx + w, rr2, t);
    }
    // ---- column phase: G^t from F^t -------------------------------------------------------
    // shifted by G^{t-1}, which the row update of this iteration used; the last block also
    // stages the residual partials
    for (int b = 0; b < nb && st == kPhaseOk; ++b) {
      const bool last = b == nb - 1;
      st = full_phase_auto<DIM, RT, CQ>(false, p, rbase + b * R, p.yc, p.CT, p.np, p.xc, p.fx, t,
                                        Gcur + b * R, buf, part, lse + b * R, &s_bad, &s_redo,
                                        &redos, p.rsx, last && t >= 2 ? p.W : 0, t, rsl);
    }
    if (st != kPhaseOk) {
      flags |= 2;
      break;
    }
    if (tid < kWave) {  // wave 0
      for (int rl = tid; rl < nr; rl += kWave) {
        const float Gn = lb2[rl] - lse[rl];
        Gprev[rl] = Gcur[rl];
        Gcur[rl] = Gn;
        slot_publish(p.gx + rbase + rl, Gn, t);
      }
    }
    // ---- stop test on the state after iteration t-1 (partials staged by the column phase)
    if (t >= 2) {
      const int lane = tid & (kWave - 1);
      float s = 0.0f;  // fixed order: every wave of every workgroup gets this very sum
      for (int v = lane; v < p.W; v += kWave) s += rsl[v];
      s = wave_sum_v(s);
      const bool fin = s == s && s < 3.0e38f;
      // tol = 0 asks for exactly max_iter iterations, even if the residual underflows to 0
      const bool conv = fin && (double)s <= p.tol2;
      if ((conv && p.tol2 > 0.0) || !fin || (int)(t - 1) >= p.max_iter) {
        err2 = s;
        converged = conv;
        if (!fin) flags |= 1;
        iters_done = (int)t - 1;
        break;
      }
    }
  }

  __syncthreads();
  for (int rl = tid; rl < nr; rl += blockDim.x) {
    p.f_out[rbase + rl] = Fprev[rl] * p.to_nat;
    p.g_out[rbase + rl] = Gprev[rl] * p.to_nat;
  }
  if (w == 0 && tid == 0) {
    p.dstats[0] = (double)iters_done;
    p.dstats[1] = (double)converged;
    p.dstats[4] = sqrt(err2);
    p.dstats[5] = (double)flags;
    p.dstats[6] = (double)redos;
    p.dstats[7] = 0.0;
  } else if (tid == 0 && flags) {
    p.dstats[5] = (double)flags;
  }
}

// Per-solve setup: pack coordinates scaled by sq = sqrt(log2(e)/eps), publish the initial
// column potential as epoch 0: 0, or g0[I mod wm] (wm = n: a full warm start; wm = m: a
// block-periodic one tiled from its first block, the second stage of Alg. 3).
template <int DIM>
__global__ void full_init_kernel(int n, int np, const float* __restrict__ x,
                                 const float* __restrict__ y, const float* __restrict__ g0,
                                 int warm, int wm, float s2, float sq, float4* __restrict__ xc,
                                 float4* __restrict__ yc, uint64_t* __restrict__ gx) {
  for (int I = blockIdx.x * blockDim.x + threadIdx.x; I < np; I += gridDim.x * blockDim.x) {
    float4 vx = make_float4(0.f, 0.f, 0.f, 0.f), vy = vx;
    if (I < n) {
      if constexpr (DIM > 0) {
        vx.x = x[(int64_t)I * DIM] * sq; vx.y = x[(int64_t)I * DIM + 1] * sq;
        vy.x = y[(int64_t)I * DIM] * sq; vy.y = y[(int64_t)I * DIM + 1] * sq;
        if constexpr (DIM == 3) { vx.z = x[(int64_t)I * 3 + 2] * sq; vy.z = y[(int64_t)I * 3 + 2] * sq; }
      }
      const float G0 = warm ? g0[I % wm] * s2 : 0.0f;
      gx[I] = (uint64_t)__float_as_uint(G0);  // epoch 0
    }
    xc[I] = vx;
    yc[I] = vy;
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

// ---- host side -------------------------------------------------------------------------
static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

static int cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return cus;
}

// (RT, CQ) variants: rows per workgroup R = (16 / CQ) * RT
struct FullVariant { int RT, CQ; };
static constexpr FullVariant kVariants[] = {{4, 1}, {4, 2}, {4, 4}, {4, 8}, {2, 8}, {1, 8}, {1, 16}};

template <int DIM, int RT, int CQ>
static const void* fk() { return (const void*)full_solver_kernel<DIM, RT, CQ>; }

static const void* pick_full_kernel(int dim, int RT, int CQ) {
#define CSOT_FK(D)                                                    \
  if (RT == 4 && CQ == 1) return fk<D, 4, 1>();                       \
  if (RT == 4 && CQ == 2) return fk<D, 4, 2>();                       \
  if (RT == 4 && CQ == 4) return fk<D, 4, 4>();                       \
  if (RT == 4 && CQ == 8) return fk<D, 4, 8>();                       \
  if (RT == 2 && CQ == 8) return fk<D, 2, 8>();                       \
  if (RT == 1 && CQ == 8) return fk<D, 1, 8>();                       \
  if (RT == 1 && CQ == 16) return fk<D, 1, 16>();                     \
  return nullptr;
  switch (dim) {
    case 0: { CSOT_FK(0) }
    case 2: { CSOT_FK(2) }
    case 3: { CSOT_FK(3) }
    default: return nullptr;
  }
#undef CSOT_FK
}

bool plan_full(const Geom& g, int hint, FullPlan* plan) {
  const int cus = cu_count();
  if (cus <= 0) return false;
  const int Wmax = hint > 0 ? hint : cus;  // one 16-wave workgroup per CU
  // smallest R (most parallelism) such that W = ceil(n / R) <= Wmax; beyond 64 Wmax rows,
  // the largest R with several row blocks per workgroup
  int best = -1;
  for (int v = (int)(sizeof(kVariants) / sizeof(kVariants[0])) - 1; v >= 0; --v) {
    const int R = (kFullWaves / kVariants[v].CQ) * kVariants[v].RT;
    if ((g.n + R - 1) / R <= Wmax) { best = v; break; }
  }
  if (best < 0) best = 0;
  const int RT = kVariants[best].RT, CQ = kVariants[best].CQ;
  const int R = (kFullWaves / CQ) * RT;
  const int blocks = (g.n + R - 1) / R;
  const int P = (blocks + Wmax - 1) / Wmax;
  if (P > kMaxRowBlocks) return false;
  const int W = (blocks + P - 1) / P;
  if (W > kFullThreads) return false;  // residual partials are staged one per thread
  const void* k = pick_full_kernel(g.dim, RT, CQ);
  if (!k) return false;
  hipFuncAttributes attr;
  if (hipFuncGetAttributes(&attr, k) != hipSuccess) return false;
  int per_cu = 0;
  // all variants have the same block size; occupancy from the kernel's own resource use
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kFullThreads, 0) != hipSuccess)
    return false;
  if (per_cu * cus < W) return false;
  plan->W = W;
  plan->R = R;
  plan->P = P;
  plan->threads = RT * 100 + CQ;  // variant code (threads per block is always kFullThreads)
  plan->lds = 0;
  return true;
}

static int full_np(int n) { return (n + kNC - 1) / kNC * kNC; }

// workspace: ctl | fx[np] | gx[np] | rsx[W] | xc[np] | yc[np] | sums[2n] | CT
size_t full_ws_bytes(const Geom& g, const FullPlan& pl) {
  const size_t np = (size_t)full_np(g.n);
  size_t b = align256(256) + 2 * align256(sizeof(uint64_t) * np) + align256(sizeof(uint64_t) * pl.W) +
             2 * align256(sizeof(float4) * np) + align256(sizeof(double) * 2 * g.n);
  if (g.dim == 0) b += align256(sizeof(float) * (size_t)g.n * np);
  return b;
}

hipError_t launch_sinkhorn_full(const Geom& g, float* f, float* gpot, double tol, int max_iter,
                                int warm, double* dstats, void* ws, const FullPlan& pl,
                                hipStream_t s, hipEvent_t* events) {
  const int np = full_np(g.n);
  char* base = static_cast<char*>(ws);
  uint32_t* ctl = reinterpret_cast<uint32_t*>(base);
  size_t off = align256(256);
  uint64_t* fx = reinterpret_cast<uint64_t*>(base + off); off += align256(sizeof(uint64_t) * np);
  uint64_t* gx = reinterpret_cast<uint64_t*>(base + off); off += align256(sizeof(uint64_t) * np);
  uint64_t* rsx = reinterpret_cast<uint64_t*>(base + off); off += align256(sizeof(uint64_t) * pl.W);
  const size_t zero_bytes = off;
  float4* xc = reinterpret_cast<float4*>(base + off); off += align256(sizeof(float4) * np);
  float4* yc = reinterpret_cast<float4*>(base + off); off += align256(sizeof(float4) * np);
  double* sums = reinterpret_cast<double*>(base + off); off += align256(sizeof(double) * 2 * g.n);
  float* CT = reinterpret_cast<float*>(base + off);

  hipError_t e = launch_zero_words(ctl, (int)(zero_bytes / 4), s);
  if (e != hipSuccess) return e;
  const float s2 = (float)(kLog2eD / g.eps);
  const float sq = (float)sqrt(kLog2eD / g.eps);
  const int ib = (np + 255) / 256 < 1024 ? (np + 255) / 256 : 1024;
  switch (g.dim) {
    case 0: hipLaunchKernelGGL(full_init_kernel<0>, dim3(ib), dim3(256), 0, s, g.n, np, g.x, g.y, gpot, warm, warm == 2 ? g.m : g.n, s2, sq, xc, yc, gx); break;
    case 2: hipLaunchKernelGGL(full_init_kernel<2>, dim3(ib), dim3(256), 0, s, g.n, np, g.x, g.y, gpot, warm, warm == 2 ? g.m : g.n, s2, sq, xc, yc, gx); break;
    case 3: hipLaunchKernelGGL(full_init_kernel<3>, dim3(ib), dim3(256), 0, s, g.n, np, g.x, g.y, gpot, warm, warm == 2 ? g.m : g.n, s2, sq, xc, yc, gx); break;
    default: return hipErrorInvalidValue;
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (g.dim == 0) {
    hipLaunchKernelGGL(transpose_kernel, dim3((g.n + 31) / 32, (g.n + 31) / 32), dim3(256), 0, s,
                       g.C, g.ldc, CT, (int64_t)np, g.n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  FullParams p;
  p.n = g.n; p.np = np; p.W = pl.W; p.R = pl.R; p.P = pl.P; p.max_iter = max_iter;
  p.s2 = s2;
  p.to_nat = (float)(g.eps * kLn2D);
  p.tol2 = tol * tol;
  p.xc = xc; p.yc = yc; p.C = g.C; p.ldc = g.ldc; p.CT = CT; p.a = g.a; p.b = g.b;
  p.f_out = f; p.g_out = gpot; p.fx = fx; p.gx = gx; p.rsx = rsx; p.ctl = ctl; p.dstats = dstats;
  void* args[] = {&p};
  const void* k = pick_full_kernel(g.dim, pl.threads / 100, pl.threads % 100);
  if (!k) return hipErrorInvalidValue;
  if (events && (e = hipEventRecord(events[0], s)) != hipSuccess) return e;
  // An ordinary launch: the plan admits no more blocks than CUs and checked that the kernel
  // fits once per CU, so on a device with no concurrent kernels every block is resident at
  // once; should one not be, the others' bounded waits end in the abort flag, not in a hang.
  e = hipLaunchKernel(k, dim3(pl.W), dim3(kFullThreads), args, 0, s);
  if (e != hipSuccess) return e;
  if (events && (e = hipEventRecord(events[1], s)) != hipSuccess) return e;

  // float64 check of the returned state
  return launch_check(g, 0, nullptr, f, gpot, g.a, g.b, sums, dstats, s);
}

}  // namespace csot
