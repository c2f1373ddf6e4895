// Cyclic Sinkhorn on the folded m x m problem (Alg. 2), one persistent launch.
//
// Log-domain updates in base 2 (F = f log2(e) / eps, G = g log2(e) / eps, L = logK log2(e)):
//   row    (eq. optimal_f_sinkhorn_logdomain):  F_i = log2 alpha_i - LSE2_j(L_ij + G_j)
//   column (log of eq. optimal_sinkhorn):       G_j = log2 beta_j  - LSE2_i(L_ij + F_i)
// starting from G = 0 (q = 1, Alg. 2 initialisation) or a warm start.
//
// Work split: workgroup w owns rows [w R, w R + R) and columns [w R, w R + R).  It keeps its
// row slab of logK and its column slab (a transposed copy) in LDS for the whole solve (natural
// log as stored; one fma per entry turns it into L), so an iteration reads no matrix data from
// memory; for m <= 512 (one row and one column per wave) each wave holds its row and column in
// registers instead, and a half-step reads only the staged potentials from LDS.  The new potentials are published as epoch-tagged 64-bit slots (value | iteration);
// each workgroup polls the m slots of the other potential until they carry the current
// iteration and stages them in LDS.  The data is its own ready flag, so there is no counter
// barrier and no cache flush; the dependency chain (F^t needs every G^{t-1}, G^t needs every
// F^t) is what keeps workgroups in step.  When the 32 workgroups of m = 512 fit on one XCD
// (blocks are dealt to XCDs round-robin, so every 8th block is launched as a real one), they
// publish through that XCD's L2.
//
// Convergence (a reading of "until convergence"): the row sums of the plan after iteration
// t-1 fall out of the row update of iteration t -- with the row shifted by its previous
// potential the shifted sum *is* that row sum -- so the residual r_i = rowsum_i - alpha_i is
// free.  Each workgroup publishes its partial sum of r_i^2 in a slot; every wave sums the W
// partials in the same order one iteration later, so all take the same stop decision without
// delaying a publication.  The returned state is (F^{t-2}, G^{t-2}) at the stop test of
// iteration t; the full-space norm is sqrt(K) ||r||_2 (every block-row of the expanded plan
// has these row sums).  At exit the workgroups exchange the returned f, g once more and
// recompute both marginal errors in float64.
#include <mutex>

#include "common.hpp"
#include "launch.hpp"

namespace csot {

constexpr int kRedThreads = 1024;        // 16 waves; one row (column) per wave at a time
constexpr int kRedWaves = kRedThreads / kWave;
constexpr int kMaxLds = 150 * 1024;
constexpr int kSweep = 4 * kWave * 2;    // elements per register sweep (two float4 per lane)
// Exchange polling of the iteration loop: loads in flight per polled slot, and the sleep
// between polls (units of 64 cycles).  The 32 workgroups of m = 512 poll the same 4 KB of
// slots, so more loads in flight lengthen the exchange (measured at n = 8192, K = 16: 2.56 us
// per iteration with two in flight and no sleep, 2.88 with three, 3.24 with four, 2.63 with
// two and a sleep of 128 cycles).
constexpr int kPollDepth = 2, kPollSleep = 0;

struct RedParams {
  int m, mp, K, W, R, max_iter, warm;
  int stride;      // launched blocks per workgroup slot (8: keep all workgroups on one XCD)
  float s2;        // log2(e) / eps
  float to_nat;    // eps ln 2
  double eps;
  double tol2;     // tol^2 / K  (compared with sum r_i^2)
  const float* logK;
  const float* alpha;
  const float* beta;
  float* f_out;
  float* g_out;
  uint64_t* fx;    // [m] F exchange slots
  uint64_t* gx;    // [m] G exchange slots
  uint64_t* rsx;   // [2][W] residual-partial slots, double-buffered by iteration parity
  uint64_t* xid;   // [W] XCD index of every workgroup (epoch 1)
  uint64_t* ffin;  // [mp] returned f (natural units) for the float64 check (epoch 1)
  uint64_t* gfin;  // [mp] returned g
  uint64_t* chk;   // [4][W] float64 check partials of every workgroup (two 32-bit halves each)
  const float* Lg;   // [m][mp] padded logK rows in device memory, or NULL: slabs held in LDS
  const float* LTg;  // [m][mp] padded logK columns (transposed), with Lg
  uint32_t* ctl;   // [0] abort flag
  double* dstats;
};

// LSE2 over a padded LDS row (length mp, a multiple of kSweep) plus `vec`, by one wave: each
// lane keeps its 8 values of a sweep in registers, the exact sweep maximum and the shifted sum
// are reduced with DPP, and sweeps are merged online.  Every lane returns the result.
__device__ __forceinline__ float wave_lse2(const float* __restrict__ row,
                                           const float* __restrict__ vec, int mp, int lane) {
  float M = kNegBig, S = 0.0f;
  for (int base = 0; base < mp; base += kSweep) {
    const int q0 = base + 4 * lane, q1 = q0 + 4 * kWave;
    const float4 l0 = *reinterpret_cast<const float4*>(row + q0);
    const float4 v0 = *reinterpret_cast<const float4*>(vec + q0);
    const float4 l1 = *reinterpret_cast<const float4*>(row + q1);
    const float4 v1 = *reinterpret_cast<const float4*>(vec + q1);
    // row holds the natural logK: base 2 by one fma per entry
    const float t[8] = {fmaf(l0.x, kLog2e, v0.x), fmaf(l0.y, kLog2e, v0.y),
                        fmaf(l0.z, kLog2e, v0.z), fmaf(l0.w, kLog2e, v0.w),
                        fmaf(l1.x, kLog2e, v1.x), fmaf(l1.y, kLog2e, v1.y),
                        fmaf(l1.z, kLog2e, v1.z), fmaf(l1.w, kLog2e, v1.w)};
    float mx = fmaxf(fmaxf(fmaxf(t[0], t[1]), fmaxf(t[2], t[3])),
                     fmaxf(fmaxf(t[4], t[5]), fmaxf(t[6], t[7])));
    mx = wave_max_v(mx);
    const float Mn = fmaxf(M, mx);
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += exp2_fast(t[k] - Mn);
    s = wave_sum_v(s);
    S = S * exp2_fast(M - Mn) + s;
    M = Mn;
  }
  return M + log2_fast(S);
}

// Shifted sum over a padded LDS row: sum_j 2^(row_j + vec_j + sh), every lane receiving it.
// With sh the row's own previous potential every term is at most the other side's marginal
// entry (the previous plan's column or row sums are exact after the other side's update), so
// the sum, the previous plan's row sum, is at most 1 and needs no maximum.
constexpr float kMinShiftedSum = 0x1p-60f;  // below this the caller redoes the row exactly

template <bool GSLAB>
__device__ __forceinline__ float wave_shifted_sum(const float* __restrict__ row,
                                                  const float* __restrict__ vec, int mp,
                                                  int lane, float sh) {
  float s = 0.0f;
  int base0 = 0;
  if constexpr (GSLAB) {
    // row in device memory: the loads of four sweeps are issued together, so that a row costs
    // one memory round trip per four sweeps rather than one per sweep
    constexpr int kG = 4;
    for (; base0 + kG * kSweep <= mp; base0 += kG * kSweep) {
      float4 l[2 * kG];
#pragma unroll
      for (int u = 0; u < kG; ++u) {
        const int q0 = base0 + u * kSweep + 4 * lane;
        l[2 * u] = *reinterpret_cast<const float4*>(row + q0);
        l[2 * u + 1] = *reinterpret_cast<const float4*>(row + q0 + 4 * kWave);
      }
#pragma unroll
      for (int u = 0; u < kG; ++u) {
        const int q0 = base0 + u * kSweep + 4 * lane;
        const float4 v0 = *reinterpret_cast<const float4*>(vec + q0);
        const float4 v1 = *reinterpret_cast<const float4*>(vec + q0 + 4 * kWave);
        const float4 l0 = l[2 * u], l1 = l[2 * u + 1];
        s += exp2_fast(fmaf(l0.x, kLog2e, v0.x + sh)) + exp2_fast(fmaf(l0.y, kLog2e, v0.y + sh)) +
             exp2_fast(fmaf(l0.z, kLog2e, v0.z + sh)) + exp2_fast(fmaf(l0.w, kLog2e, v0.w + sh)) +
             exp2_fast(fmaf(l1.x, kLog2e, v1.x + sh)) + exp2_fast(fmaf(l1.y, kLog2e, v1.y + sh)) +
             exp2_fast(fmaf(l1.z, kLog2e, v1.z + sh)) + exp2_fast(fmaf(l1.w, kLog2e, v1.w + sh));
      }
    }
  }
  for (int base = base0; base < mp; base += kSweep) {
    const int q0 = base + 4 * lane, q1 = q0 + 4 * kWave;
    const float4 l0 = *reinterpret_cast<const float4*>(row + q0);
    const float4 v0 = *reinterpret_cast<const float4*>(vec + q0);
    const float4 l1 = *reinterpret_cast<const float4*>(row + q1);
    const float4 v1 = *reinterpret_cast<const float4*>(vec + q1);
    s += exp2_fast(fmaf(l0.x, kLog2e, v0.x + sh)) + exp2_fast(fmaf(l0.y, kLog2e, v0.y + sh)) +
         exp2_fast(fmaf(l0.z, kLog2e, v0.z + sh)) + exp2_fast(fmaf(l0.w, kLog2e, v0.w + sh)) +
         exp2_fast(fmaf(l1.x, kLog2e, v1.x + sh)) + exp2_fast(fmaf(l1.y, kLog2e, v1.y + sh)) +
         exp2_fast(fmaf(l1.z, kLog2e, v1.z + sh)) + exp2_fast(fmaf(l1.w, kLog2e, v1.w + sh));
  }
  return wave_sum_v(s);
}

// One potential update by one wave: the new potential lm - LSE2_j(row_j + vec_j) and the
// previous plan's marginal sum.  Shifted by the previous potential `prev` when `shifted`,
// falling back to the exact running-maximum form when the shifted sum is out of range.
template <bool GSLAB>
__device__ __forceinline__ float wave_update(const float* __restrict__ row,
                                             const float* __restrict__ vec, int mp, int lane,
                                             float lm, float prev, bool shifted, float* sum_out) {
  if (shifted) {
    const float S = wave_shifted_sum<GSLAB>(row, vec, mp, lane, prev);
    if (S >= kMinShiftedSum && S < INFINITY) {
      *sum_out = S;
      return lm - log2_fast(S) + prev;
    }
  }
  const float Fn = lm - wave_lse2(row, vec, mp, lane);
  *sum_out = -1.0f;  // not available: the caller uses the potential difference
  return Fn;
}

// The same update when the padded row is one sweep (mp == kSweep) held in registers: l0, l1
// are this lane's 8 entries of the row (natural logK), as the LDS forms read them.
__device__ __forceinline__ float wave_update_reg(const float4& l0, const float4& l1,
                                                 const float* __restrict__ vec, int lane,
                                                 float lm, float prev, bool shifted,
                                                 float* sum_out) {
  const int q0 = 4 * lane, q1 = q0 + 4 * kWave;
  const float4 v0 = *reinterpret_cast<const float4*>(vec + q0);
  const float4 v1 = *reinterpret_cast<const float4*>(vec + q1);
  const float t[8] = {fmaf(l0.x, kLog2e, v0.x), fmaf(l0.y, kLog2e, v0.y),
                      fmaf(l0.z, kLog2e, v0.z), fmaf(l0.w, kLog2e, v0.w),
                      fmaf(l1.x, kLog2e, v1.x), fmaf(l1.y, kLog2e, v1.y),
                      fmaf(l1.z, kLog2e, v1.z), fmaf(l1.w, kLog2e, v1.w)};
  if (shifted) {
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += exp2_fast(t[k] + prev);
    const float S = wave_sum_v(s);
    if (S >= kMinShiftedSum && S < INFINITY) {
      *sum_out = S;
      return lm - log2_fast(S) + prev;
    }
  }
  float mx = fmaxf(fmaxf(fmaxf(t[0], t[1]), fmaxf(t[2], t[3])),
                   fmaxf(fmaxf(t[4], t[5]), fmaxf(t[6], t[7])));
  mx = fmaxf(kNegBig, wave_max_v(mx));
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += exp2_fast(t[k] - mx);
  s = wave_sum_v(s);
  *sum_out = -1.0f;
  return lm - (mx + log2_fast(s));
}

// GSLAB: the slabs are read from the padded copies in device memory (large m); otherwise they
// are loaded into LDS once.  A template parameter, so that either way the compiler knows the
// slabs' address space (LDS reads stay ds_read, not flat loads).
template <bool GSLAB>
__global__ void __launch_bounds__(kRedThreads) reduced_solver_kernel(RedParams p) {
  extern __shared__ float4 lds4[];
  float* lds = reinterpret_cast<float*>(lds4);
  const int R = p.R, mp = p.mp, m = p.m;
  // slabs in LDS, or (large m) read from the padded copies in device memory every half-step
  constexpr bool gslab = GSLAB;
  const size_t slab = gslab ? 0 : (size_t)R * mp;
  float* Ls_l = lds;                    // [R][mp] row slab
  float* LTs_l = Ls_l + slab;           // [R][mp] column slab (transposed)
  float* VsG = LTs_l + slab;            // [mp] staged G (read by row updates)
  float* VsF = VsG + mp;                // [mp] staged F (read by column updates)
  float* la2 = VsF + mp;                // [R] log2 alpha (my rows)
  float* lb2 = la2 + R;                 // [R] log2 beta (my columns)
  float* av = lb2 + R;                  // [R] alpha (my rows)
  float* Fcur = av + R;                 // [R] F^t
  float* Fprev = Fcur + R;              // [R] F^{t-1}
  float* Gcur = Fprev + R;              // [R] G^t
  float* Gprev = Gcur + R;              // [R] G^{t-1}
  float* Fold = Gprev + R;              // [R] F^{t-2} while the stop test of t-1 runs
  float* rsv = Fold + R;                // [W] residual partials of every workgroup
  __shared__ float wsum[kRedWaves];
  __shared__ int s_bad;
  __shared__ int s_mixed;

  if (blockIdx.x % p.stride) return;  // placeholder block: frees its CU at once
  const int w = blockIdx.x / p.stride;
  const int r0 = w * R;
  const float* Ls = GSLAB ? p.Lg + (size_t)r0 * mp : Ls_l;
  const float* LTs = GSLAB ? p.LTg + (size_t)r0 * mp : LTs_l;
  const int nr = max(0, min(R, m - r0));  // rows (= columns) this workgroup owns
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wv = tid / kWave;
  uint32_t* abort_flag = p.ctl;

  // announce this workgroup's XCD before the slab load, so that the check after it rarely waits
  if (p.stride > 1 && tid == 0) slot_publish(p.xid + w, __uint_as_float(xcc_id()), 1u);

  // ---- load the slabs (once) ------------------------------------------------------------
  // Row slab Ls[rl][j] = logK[r0 + rl][j], column slab LTs[cl][i] = logK[i][r0 + cl], -inf in
  // the padding.  With m and R multiples of 4 both read float4 (four consecutive columns);
  // 8 loads in flight per thread before the first store (one memory round trip per 8).
  constexpr int kLd = 8;
  if constexpr (GSLAB) {
    // nothing to load: the padded copies are read in place
  } else if ((m & 3) == 0 && (R & 3) == 0 && (reinterpret_cast<uintptr_t>(p.logK) & 15) == 0) {
    const float4 ninf = make_float4(-INFINITY, -INFINITY, -INFINITY, -INFINITY);
    const int q4 = mp / 4, r4 = R / 4;
    const int nrow = R * q4, ncol = mp * r4;  // quads of the row slab, of the column slab
    for (int e0 = tid; e0 < nrow + ncol; e0 += kLd * blockDim.x) {
      float4 v[kLd];
#pragma unroll
      for (int u = 0; u < kLd; ++u) {
        const int e = e0 + u * blockDim.x;
        v[u] = ninf;
        if (e < nrow) {
          const int rl = e / q4, j = 4 * (e - rl * q4);
          if (rl < nr && j < m) v[u] = *reinterpret_cast<const float4*>(p.logK + (int64_t)(r0 + rl) * m + j);
        } else if (e < nrow + ncol) {
          const int ec = e - nrow;
          const int i = ec / r4, cl = 4 * (ec - i * r4);
          if (i < m && cl < nr) {
            v[u] = *reinterpret_cast<const float4*>(p.logK + (int64_t)i * m + r0 + cl);
            if (cl + 1 >= nr) v[u].y = -INFINITY;
            if (cl + 2 >= nr) v[u].z = -INFINITY;
            if (cl + 3 >= nr) v[u].w = -INFINITY;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kLd; ++u) {
        const int e = e0 + u * blockDim.x;
        if (e < nrow) {
          *reinterpret_cast<float4*>(Ls_l + 4 * (size_t)e) = v[u];  // natural log
        } else if (e < nrow + ncol) {
          const int ec = e - nrow;
          const int i = ec / r4, cl = 4 * (ec - i * r4);
          LTs_l[(size_t)cl * mp + i] = v[u].x;
          LTs_l[(size_t)(cl + 1) * mp + i] = v[u].y;
          LTs_l[(size_t)(cl + 2) * mp + i] = v[u].z;
          LTs_l[(size_t)(cl + 3) * mp + i] = v[u].w;
        }
      }
    }
  } else {
    for (int e0 = tid; e0 < R * mp; e0 += kLd * blockDim.x) {
      float v[kLd], vt[kLd];
#pragma unroll
      for (int u = 0; u < kLd; ++u) {
        const int e = e0 + u * blockDim.x;
        const int rl = e / mp, j = e - rl * mp;
        v[u] = (e < R * mp && rl < nr && j < m) ? p.logK[(int64_t)(r0 + rl) * m + j] : -INFINITY;
        const int i = e / R, cl = e - i * R;  // consecutive threads read consecutive columns
        vt[u] = (e < R * mp && cl < nr && i < m) ? p.logK[(int64_t)i * m + r0 + cl] : -INFINITY;
      }
#pragma unroll
      for (int u = 0; u < kLd; ++u) {
        const int e = e0 + u * blockDim.x;
        if (e < R * mp) {
          Ls_l[e] = v[u];  // natural log
          const int i = e / R, cl = e - i * R;
          LTs_l[(size_t)cl * mp + i] = vt[u];
        }
      }
    }
  }
  for (int rl = tid; rl < R; rl += blockDim.x) {
    const bool ok = rl < nr;
    la2[rl] = ok ? log2f(p.alpha[r0 + rl]) : 0.0f;
    lb2[rl] = ok ? log2f(p.beta[r0 + rl]) : 0.0f;
    av[rl] = ok ? p.alpha[r0 + rl] : 0.0f;
    Gcur[rl] = ok && p.warm ? p.g_out[r0 + rl] * p.s2 : 0.0f;
    Gprev[rl] = Gcur[rl];
    Fcur[rl] = 0.0f;
    Fprev[rl] = 0.0f;
    Fold[rl] = 0.0f;
  }
  for (int j = tid; j < mp; j += blockDim.x) {
    VsG[j] = (j < m && p.warm) ? p.g_out[j] * p.s2 : 0.0f;
    VsF[j] = 0.0f;
  }
  if (tid == 0) {
    s_bad = 0;
    s_mixed = 0;
  }
  __syncthreads();

  int iters_done = 0, converged = 0, flags = 0;
  float err2 = 0.0f;

  // A row of one sweep and at most one row (column) per wave: each wave keeps its row and its
  // column of logK in registers for the whole solve, so that a half-step reads only the
  // staged potentials from LDS.
  const bool reg = !GSLAB && mp == kSweep && nr <= kRedWaves;
  float4 lr0 = {}, lr1 = {}, lc0 = {}, lc1 = {};
  if (reg && wv < nr) {
    const int q0 = 4 * lane, q1 = q0 + 4 * kWave;
    lr0 = *reinterpret_cast<const float4*>(Ls + (size_t)wv * mp + q0);
    lr1 = *reinterpret_cast<const float4*>(Ls + (size_t)wv * mp + q1);
    lc0 = *reinterpret_cast<const float4*>(LTs + (size_t)wv * mp + q0);
    lc1 = *reinterpret_cast<const float4*>(LTs + (size_t)wv * mp + q1);
  }

  // When the launch placed every workgroup on one XCD (stride 8), confirm it: then the
  // potentials can be published through that XCD's L2 alone (slot_publish_local), which
  // halves the exchange latency.  Otherwise every publication is agent-scope.
  bool local_pub = false;
  if (p.stride > 1) {
    const uint32_t me = xcc_id();
    for (int v = tid; v < p.W; v += blockDim.x) {
      uint64_t x = slot_load(p.xid + v);
      if (!slot_wait(p.xid + v, x, 1u, abort_flag)) s_bad = 1;
      else if (__float_as_uint(slot_value(x)) != me) s_mixed = 1;
    }
    __syncthreads();
    local_pub = !s_mixed;
  }
  auto publish = [&](uint64_t* slot, float v, uint32_t epoch) {
    if (local_pub) slot_publish_local(slot, v, epoch);
    else slot_publish(slot, v, epoch);
  };
  // read once, before any wave can reach an exchange (which may set s_bad again)
  const bool started = s_bad == 0;
  if (!started) flags |= 2;

  // Iteration t: row update (F^t from G^{t-1}; the row sums of the state after t-1 fall out of
  // it), publication of F^t, the stop test on the state after t-2 whose residual partials
  // arrived with G^{t-1} (every wave evaluates it from the same staged values, so no barrier
  // is needed and it never delays a publication), exchange of F^t, publication of this
  // workgroup's residual partial of iteration t, column update (G^t), exchange of G^t together
  // with the residual partials of iteration t.  The two staged potentials have buffers of
  // their own, so the two exchanges are the only barriers of an iteration.
  for (uint32_t t = 1; started; ++t) {
    // ---- row update ----------------------------------------------------------------------
    float racc = 0.0f;
    for (int rl = wv; rl < nr; rl += kRedWaves) {
      float S;
      const float Fo = Fcur[rl];
      const float Fn =
          reg ? wave_update_reg(lr0, lr1, VsG, lane, la2[rl], Fo, t >= 2, &S)
              : wave_update<GSLAB>(Ls + (size_t)rl * mp, VsG, mp, lane, la2[rl], Fo, t >= 2, &S);
      if (lane == 0) {
        publish(p.fx + r0 + rl, Fn, t);  // first: the other workgroups wait for it
        if (t >= 2) {
          // residual of the state after t-1: its row sum minus alpha
          const float rr = S >= 0.0f ? S - av[rl] : scaled_exp2m1(av[rl], Fo - Fn);
          racc += rr * rr;
        }
        Fold[rl] = Fprev[rl];
        Fprev[rl] = Fo;
        Fcur[rl] = Fn;
      }
    }
    if (lane == 0) wsum[wv] = racc;

    // ---- stop test on the state after iteration t-2 (its residual came with G^{t-1}) -------
    if (t >= 3) {
      float s = 0.0f;  // fixed-order reduction: every wave of every workgroup gets this sum
      for (int v = lane; v < p.W; v += kWave) s += rsv[v];
      s = wave_sum_v(s);
      err2 = s;
      const bool fin = s == s && s < 3.0e38f;
      converged = fin && (double)s <= p.tol2;
      if (!fin) flags |= 1;
      // tol = 0 asks for exactly max_iter iterations, even if the residual underflows
      if ((converged && p.tol2 > 0.0) || !fin || (int)(t - 2) >= p.max_iter) {
        iters_done = (int)t - 2;
        break;
      }
    }

    // ---- exchange F^t (barrier), residual partial of iteration t, column update -----------
    if (!stage_slots<kPollSleep, kPollDepth>(p.fx, m, mp, t, VsF, nullptr, 0, 0, nullptr, abort_flag, &s_bad)) {
      flags |= 2;
      break;
    }
    if (wv == 0 && t >= 2) {
      float s = lane < kRedWaves ? wsum[lane] : 0.0f;
      s = wave_sum_v(s);
      if (lane == 0) publish(p.rsx + (t & 1u) * p.W + w, s, t);
    }
    for (int cl = wv; cl < nr; cl += kRedWaves) {
      float S;
      const float Go = Gcur[cl];
      const float Gn =
          reg ? wave_update_reg(lc0, lc1, VsF, lane, lb2[cl], Go, true, &S)
              : wave_update<GSLAB>(LTs + (size_t)cl * mp, VsF, mp, lane, lb2[cl], Go, true, &S);
      if (lane == 0) {
        publish(p.gx + r0 + cl, Gn, t);
        Gprev[cl] = Go;
        Gcur[cl] = Gn;
      }
    }

    // ---- exchange G^t and the residual partials of iteration t (barrier) ----------------------
    // A workgroup that is one iteration ahead may already publish its next residual partial
    // while this one still polls; the parity buffers keep the two apart.
    const int nres = t >= 2 ? p.W : 0;
    if (!stage_slots<kPollSleep, kPollDepth>(p.gx, m, mp, t, VsG, p.rsx + (t & 1u) * p.W, nres, t, rsv, abort_flag,
                     &s_bad)) {
      flags |= 2;
      break;
    }
  }

  // ---- outputs: the state after iteration iters_done = t - 2, i.e. (F^{t-2}, G^{t-2}) -----
  // At the stop test of iteration t the row update of t has run (Fcur = F^t, Fprev = F^{t-1},
  // Fold = F^{t-2}) and the column update of t has not (Gcur = G^{t-1}, Gprev = G^{t-2}).
  __syncthreads();
  for (int rl = tid; rl < nr; rl += blockDim.x) {
    const float fo = Fold[rl] * p.to_nat, go = Gprev[rl] * p.to_nat;
    p.f_out[r0 + rl] = fo;
    p.g_out[r0 + rl] = go;
    publish(p.ffin + r0 + rl, fo, 1u);
    publish(p.gfin + r0 + rl, go, 1u);
  }
  if (w == 0 && tid == 0) {
    p.dstats[0] = (double)iters_done;
    p.dstats[1] = (double)converged;
    p.dstats[4] = sqrt((double)p.K * (double)err2);
    p.dstats[5] = (double)flags;
    p.dstats[6] = 0.0;
    p.dstats[7] = local_pub ? 1.0 : 0.0;
  } else if (tid == 0 && flags) {
    p.dstats[5] = (double)flags;
  }

  // ---- float64 check of the returned state: full-space L2 marginal errors --------------------
  // Every workgroup stages all returned f and g (natural units, as written) and sums its own
  // rows and columns of the reduced plan T_ij = exp(logK_ij + (f_i + g_j) / eps) from the
  // stored logK in float64; it publishes its two squared-residual partials (each as two 32-bit
  // halves in epoch-tagged slots), and workgroup 0 sums all of them in a fixed order and
  // writes sqrt(K sum).
  const bool staged = stage_slots(p.ffin, m, mp, 1u, VsF, p.gfin, m, 1u, VsG, abort_flag, &s_bad);
  const double inv_eps = 1.0 / p.eps;
  double part_r = 0.0, part_c = 0.0;
  if (staged) {
    for (int q = wv; q < 2 * nr; q += kRedWaves) {
      const bool row = q < nr;
      const int o = r0 + (row ? q : q - nr);         // own row i or own column j
      const double po = (double)(row ? VsF[o] : VsG[o]);
      const float* opot = row ? VsG : VsF;
      const float* slab = (row ? Ls : LTs) + (size_t)(o - r0) * mp;  // stored logK, natural
      // four independent float64 exponentials in flight per lane (one wave per SIMD here)
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int b = lane;
      for (; b + 3 * kWave < m; b += 4 * kWave) {
        s0 += exp((double)slab[b] + (po + (double)opot[b]) * inv_eps);
        s1 += exp((double)slab[b + kWave] + (po + (double)opot[b + kWave]) * inv_eps);
        s2 += exp((double)slab[b + 2 * kWave] + (po + (double)opot[b + 2 * kWave]) * inv_eps);
        s3 += exp((double)slab[b + 3 * kWave] + (po + (double)opot[b + 3 * kWave]) * inv_eps);
      }
      for (; b < m; b += kWave) s0 += exp((double)slab[b] + (po + (double)opot[b]) * inv_eps);
      const double sum = wave_sum_d((s0 + s1) + (s2 + s3));
      const double d = sum - (double)(row ? p.alpha[o] : p.beta[o]);
      if (lane == 0) {
        if (row) part_r += d * d;
        else part_c += d * d;
      }
    }
  }
  __shared__ double s_acc[2 * kRedWaves];
  if (lane == 0) {
    s_acc[wv] = part_r;
    s_acc[kRedWaves + wv] = part_c;
  }
  __syncthreads();
  if (tid < 2) {
    double v = 0.0;
    for (int k = 0; k < kRedWaves; ++k) v += s_acc[tid * kRedWaves + k];
    const uint64_t bits = (uint64_t)__double_as_longlong(v);
    publish(p.chk + (2 * tid) * p.W + w, __uint_as_float((uint32_t)(bits >> 32)), 1u);
    publish(p.chk + (2 * tid + 1) * p.W + w, __uint_as_float((uint32_t)bits), 1u);
  }
  if (w == 0 && wv == 0) {
    double r = 0.0, c = 0.0;
    bool ok = staged;
    for (int v = lane; v < p.W; v += kWave) {
      uint64_t h[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) h[k] = slot_load(p.chk + k * p.W + v);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (ok) ok = slot_wait(p.chk + k * p.W + v, h[k], 1u, abort_flag);
      r += __longlong_as_double((long long)(((uint64_t)__float_as_uint(slot_value(h[0])) << 32) |
                                            __float_as_uint(slot_value(h[1]))));
      c += __longlong_as_double((long long)(((uint64_t)__float_as_uint(slot_value(h[2])) << 32) |
                                            __float_as_uint(slot_value(h[3]))));
    }
    r = wave_sum_d(r);
    c = wave_sum_d(c);
    ok = __all(ok) && s_bad == 0;  // s_bad: an abort seen by this workgroup's exchanges
    if (lane == 0) {
      p.dstats[2] = ok ? sqrt((double)p.K * r) : NAN;
      p.dstats[3] = ok ? sqrt((double)p.K * c) : NAN;
    }
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

static size_t reduced_lds_bytes(int R, int mp, int W, bool gslab = false) {
  return sizeof(float) * ((gslab ? 0 : (size_t)2 * R * mp) + 2 * (size_t)mp + 9 * (size_t)R + W) +
         16;
}

// Padded copies of logK for the large-m mode: Lg[i][j] = logK[i][j], LTg[j][i] = logK[i][j],
// rows of mp floats with -inf beyond m.  32 x 32 tiles through LDS; the grid covers mp x mp so
// that the padding of both copies is written too.
__global__ void __launch_bounds__(256)
    pad_slabs_kernel(const float* __restrict__ logK, int m, int mp, float* __restrict__ Lg,
                     float* __restrict__ LTg) {
  __shared__ float tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;  // columns j, rows i of logK
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int i = by + k, j = bx + tx;
    const float v = (i < m && j < m) ? logK[(int64_t)i * m + j] : -INFINITY;
    if (i < m) Lg[(int64_t)i * mp + j] = v;
    tile[k][tx] = v;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int j = bx + k, i = by + tx;  // LTg[j][i] = logK[i][j]
    if (j < m) LTg[(int64_t)j * mp + i] = tile[tx][k];
  }
}

static int reduced_mp(int m) { return (m + kSweep - 1) / kSweep * kSweep; }

bool plan_reduced(int m, int hint, ReducedPlan* plan) {
  const int cus = device_cu_count();
  if (cus <= 0) return false;
  const int mp = reduced_mp(m);
  int W = hint;
  if (W <= 0) {
    // about 16 rows per workgroup (one per wave), at most one workgroup per CU; at m = 512
    // the 32 workgroups then fit on one XCD
    W = (m + kRedWaves - 1) / kRedWaves;
    if (W < 1) W = 1;
    if (W > cus) W = cus;
  }
  if (W > m) W = m;
  int R = (m + W - 1) / W;
  W = (m + R - 1) / R;  // no empty workgroups
  size_t lds = reduced_lds_bytes(R, mp, W);
  // slabs too large for LDS: fewer rows per workgroup, more workgroups.  R drops by at least
  // one per step (W = ceil(m / (R - 1)) gives ceil(m / W) <= R - 1), so the loop ends.
  while (lds > (size_t)kMaxLds && R > 1) {
    --R;
    W = (m + R - 1) / R;
    if (W > cus) break;
    R = (m + W - 1) / W;  // no empty workgroups
    lds = reduced_lds_bytes(R, mp, W);
  }
  bool gslab = false;
  if (lds > (size_t)kMaxLds || W > cus) {
    // large m: the slabs stay in device memory (padded copies, read every half-step from the
    // L2 / last-level cache) and LDS holds only the staged potentials
    gslab = true;
    W = hint > 0 ? hint : (m + kRedWaves - 1) / kRedWaves;
    if (W > cus) W = cus;
    if (W > m) W = m;
    R = (m + W - 1) / W;
    W = (m + R - 1) / R;
    lds = reduced_lds_bytes(R, mp, W, true);
    if (lds > (size_t)kMaxLds) return false;
  }
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute((const void*)reduced_solver_kernel<false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds) != hipSuccess ||
        hipFuncSetAttribute((const void*)reduced_solver_kernel<true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds) != hipSuccess)
      return false;
    attr_set = true;
  }
  // co-residency: the persistent launch needs all W workgroups resident at once
  int per_cu = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, gslab ? reduced_solver_kernel<true> : reduced_solver_kernel<false>, kRedThreads,
      lds);
  // keep every workgroup on one XCD (blocks are dealt to the 8 XCDs round-robin) when the
  // placeholder blocks still fit in one co-resident grid: polls then stay within one L2
  const int stride = (8 * W <= cus && cus % 8 == 0) ? 8 : 1;
  if (e != hipSuccess || per_cu * cus < W * stride) return false;
  plan->stride = stride;
  plan->gslab = gslab ? 1 : 0;
  plan->W = W;
  plan->R = R;
  plan->threads = kRedThreads;
  plan->lds = lds;
  return true;
}

// workspace: ctl[64 words] | fx[mp] | gx[mp] | rsx[2W] | xid[W] | ffin[mp] | gfin[mp] | chk[4W]
// (64-bit slots)
static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

static size_t slots_bytes(int m, int W) {
  return align256(256) + 4 * align256(sizeof(uint64_t) * reduced_mp(m)) +
         align256(sizeof(uint64_t) * 2 * W) + align256(sizeof(uint64_t) * W) +
         align256(sizeof(uint64_t) * 4 * W);
}

size_t reduced_ws_bytes(int m, const ReducedPlan& p) {
  const size_t slabs = p.gslab ? 2 * align256(sizeof(float) * (size_t)m * reduced_mp(m)) : 0;
  return slots_bytes(m, p.W) + slabs;
}

hipError_t launch_sinkhorn_reduced(int m, int K, double eps, const float* logK,
                                   const float* alpha, const float* beta, float* f, float* g,
                                   double tol, int max_iter, int warm, double* dstats,
                                   void* ws, const ReducedPlan& pl, hipStream_t s,
                                   hipEvent_t* events) {
  const int mp = reduced_mp(m);
  char* base = static_cast<char*>(ws);
  uint32_t* ctl = reinterpret_cast<uint32_t*>(base);
  size_t off = align256(256);
  uint64_t* fx = reinterpret_cast<uint64_t*>(base + off); off += align256(sizeof(uint64_t) * mp);
  uint64_t* gx = reinterpret_cast<uint64_t*>(base + off); off += align256(sizeof(uint64_t) * mp);
  uint64_t* rsx = reinterpret_cast<uint64_t*>(base + off); off += align256(sizeof(uint64_t) * 2 * pl.W);
  uint64_t* xid = reinterpret_cast<uint64_t*>(base + off); off += align256(sizeof(uint64_t) * pl.W);
  uint64_t* ffin = reinterpret_cast<uint64_t*>(base + off); off += align256(sizeof(uint64_t) * mp);
  uint64_t* gfin = reinterpret_cast<uint64_t*>(base + off); off += align256(sizeof(uint64_t) * mp);
  uint64_t* chk = reinterpret_cast<uint64_t*>(base + off); off += align256(sizeof(uint64_t) * 4 * pl.W);
  const size_t slots_end = off;
  float* Lg = nullptr;
  float* LTg = nullptr;
  if (pl.gslab) {
    Lg = reinterpret_cast<float*>(base + off); off += align256(sizeof(float) * (size_t)m * mp);
    LTg = reinterpret_cast<float*>(base + off); off += align256(sizeof(float) * (size_t)m * mp);
  }

  // epochs start at 1, so zeroed slots are never mistaken for current ones
  hipError_t e = launch_zero_words(ctl, (int)(slots_end / 4), s);
  if (e != hipSuccess) return e;
  if (pl.gslab) {
    hipLaunchKernelGGL(pad_slabs_kernel, dim3(mp / 32, mp / 32), dim3(256), 0, s, logK, m, mp,
                       Lg, LTg);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }

  RedParams p;
  p.m = m; p.mp = mp; p.K = K; p.W = pl.W; p.R = pl.R; p.max_iter = max_iter; p.warm = warm;
  p.stride = pl.stride;
  p.s2 = (float)(kLog2eD / eps);
  p.to_nat = (float)(eps * kLn2D);
  p.tol2 = tol * tol / (double)K;
  p.logK = logK; p.alpha = alpha; p.beta = beta; p.f_out = f; p.g_out = g;
  p.fx = fx; p.gx = gx; p.rsx = rsx; p.xid = xid; p.ffin = ffin; p.gfin = gfin; p.chk = chk; p.ctl = ctl;
  p.Lg = Lg; p.LTg = LTg;
  p.dstats = dstats;
  p.eps = eps;
  void* args[] = {&p};
  if (events && (e = hipEventRecord(events[0], s)) != hipSuccess) return e;
  // An ordinary launch: the plan admits at most one block per CU and no more blocks than CUs,
  // so on a device with no concurrent kernels every block is resident at once (the cooperative
  // launch API guarantees the same but adds ~10 us of dispatch overhead on each side).  Should a
  // block not be resident, the others' bounded waits end in the abort flag, not in a hang.
  auto kern = pl.gslab ? reduced_solver_kernel<true> : reduced_solver_kernel<false>;
  hipLaunchKernelGGL(kern, dim3(pl.W * pl.stride), dim3(pl.threads),
                     (unsigned)pl.lds, s, p);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (events && (e = hipEventRecord(events[1], s)) != hipSuccess) return e;

  return hipSuccess;
}

// ---- allocation-free entry: fixed scratch in device memory ---------------------------------
// One copy per device, held until the process ends.  Host code never passes `scratch` itself
// (in host code the name is a host-side stand-in, not a device address): the device address
// comes from hipGetSymbolAddress, fetched once per device with that device current.
static __device__ __align__(256) unsigned char scratch[kReducedScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t reduced_scratch(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace csot
