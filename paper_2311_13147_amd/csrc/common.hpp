// Device helpers shared by the csot kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace csot {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr double kLog2eD = 1.4426950408889634074;
constexpr double kLn2D = 0.69314718055994530942;
constexpr float kNegBig = -1.0e30f;  // finite "minus infinity" for running maxima
constexpr int kWave = 64;

// Read-only float data in device (global) memory.  Pointers taken from a descriptor in memory
// are generic to the compiler, which then emits flat loads with 64-bit address arithmetic;
// the cast lets it use global loads with 32-bit offsets from a scalar base.
typedef __attribute__((address_space(1))) const float gcfloat;
__device__ __forceinline__ gcfloat* as_global(const float* p) { return (gcfloat*)p; }

// 2^x and log2(x) on the transcendental unit (v_exp_f32 / v_log_f32, 1 ulp).
__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float log2_fast(float x) { return __builtin_amdgcn_logf(x); }

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Cross-lane moves on the VALU (DPP) within a row of 16 lanes: lane i reads lane i^1, i^2,
// the mirror within its half-row (7 - i) and the mirror within its row (15 - i).  Applied in
// that order, a reduction leaves every lane of the row with the row's result.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141; // row_half_mirror
constexpr int kDppMirror = 0x140;     // row_mirror

// Merge of two (max, sum) log-sum-exp partials in base 2: value = M + log2(S).
__device__ __forceinline__ void lse_merge(float& M, float& S, float M2, float S2) {
  const float Mn = fmaxf(M, M2);
  S = S * exp2_fast(M - Mn) + S2 * exp2_fast(M2 - Mn);
  M = Mn;
}

// Wave-wide sum with every lane receiving the result: DPP inside rows of 16 lanes, a swizzle
// across rows (xor 16), then the two half-waves combined through lanes 0 and 32.
__device__ __forceinline__ float wave_sum_all(float v) {
  v += dpp_f32<kDppXor1>(v);
  v += dpp_f32<kDppXor2>(v);
  v += dpp_f32<kDppHalfMirror>(v);
  v += dpp_f32<kDppMirror>(v);
  v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
  const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  return a + b;
}

// Wave-wide sum / max on the vector unit alone, every lane receiving the bitwise-identical
// result: DPP inside rows of 16 lanes, then v_permlane16_swap (row pairs) and
// v_permlane32_swap (the two halves).  Each lane combines the two operands in the same order,
// so all lanes (and all waves holding the same inputs) agree exactly.
__device__ __forceinline__ float swap_sum16(float v) {
  const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(a[0]) + __uint_as_float(a[1]);
}
__device__ __forceinline__ float swap_sum32(float v) {
  const auto a = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(a[0]) + __uint_as_float(a[1]);
}
__device__ __forceinline__ float wave_sum_v(float v) {
  v += dpp_f32<kDppXor1>(v);
  v += dpp_f32<kDppXor2>(v);
  v += dpp_f32<kDppHalfMirror>(v);
  v += dpp_f32<kDppMirror>(v);
  return swap_sum32(swap_sum16(v));
}
__device__ __forceinline__ float wave_max_v(float v) {
  v = fmaxf(v, dpp_f32<kDppXor1>(v));
  v = fmaxf(v, dpp_f32<kDppXor2>(v));
  v = fmaxf(v, dpp_f32<kDppHalfMirror>(v));
  v = fmaxf(v, dpp_f32<kDppMirror>(v));
  auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = fmaxf(__uint_as_float(a[0]), __uint_as_float(a[1]));
  a = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return fmaxf(__uint_as_float(a[0]), __uint_as_float(a[1]));
}

// ---- float64 cross-lane moves (each 32-bit half moved on its own) ----------------------
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// v_permlane32_swap / v_permlane16_swap of the pair (a, b): afterwards a + b is, in lanes whose
// bit 5 (bit 4) is clear, a + partner's a and, in the others, partner's b + b (partner = lane
// with that bit flipped).
__device__ __forceinline__ void swap32_f64(double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a),
                                                   (unsigned)__double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a),
                                                   (unsigned)__double2hiint(b), false, false);
  a = __hiloint2double((int)hi[0], (int)lo[0]);
  b = __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ void swap16_f64(double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a),
                                                   (unsigned)__double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a),
                                                   (unsigned)__double2hiint(b), false, false);
  a = __hiloint2double((int)hi[0], (int)lo[0]);
  b = __hiloint2double((int)hi[1], (int)lo[1]);
}

// Wave-wide float64 sum on the vector unit, every lane receiving the result.
__device__ __forceinline__ double wave_sum_all_d(double v) {
  v += dpp_f64<kDppXor1>(v);
  v += dpp_f64<kDppXor2>(v);
  v += dpp_f64<kDppHalfMirror>(v);
  v += dpp_f64<kDppMirror>(v);
  double w = v;
  swap16_f64(v, w);
  v += w;
  w = v;
  swap32_f64(v, w);
  return v + w;
}

constexpr int ilog2_ceil(int v) {
  int s = 0;
  while ((1 << s) < v) ++s;
  return s;
}

// Reduce-scatter of NV = 2^S float64 values over groups of 2^B consecutive lanes (B <= 6):
// halving steps over lane bits B-1 .. 0 while more than one value is left, then plain sums
// over the remaining bits.  On return lane l holds, in v[0 .. L), L = 2^max(S - B, 0), the
// group totals of values (l mod 2^B) >> max(B - S, 0) ... : value index
//   (l mod 2^B) * L + j            when S >= B,
//   (l mod 2^B) >> (B - S)         (j = 0) when S < B.
template <int BIT, int L, int NV>
__device__ __forceinline__ void rs_step(double (&v)[NV], int lane) {
  if constexpr (BIT == 5 || BIT == 4) {
    if constexpr (L > 1) {
#pragma unroll
      for (int q = 0; q < L / 2; ++q) {
        if constexpr (BIT == 5) swap32_f64(v[q], v[q + L / 2]);
        else swap16_f64(v[q], v[q + L / 2]);
        v[q] += v[q + L / 2];
      }
    } else {
      double w = v[0];
      if constexpr (BIT == 5) swap32_f64(v[0], w);
      else swap16_f64(v[0], w);
      v[0] += w;
    }
  } else {
    constexpr int CTRL = BIT == 3 ? kDppMirror : BIT == 2 ? kDppHalfMirror : BIT == 1 ? kDppXor2 : kDppXor1;
    if constexpr (L > 1) {
      const bool hi = (lane & (1 << BIT)) != 0;
#pragma unroll
      for (int q = 0; q < L / 2; ++q) {
        const double keep = hi ? v[q + L / 2] : v[q];
        const double send = hi ? v[q] : v[q + L / 2];
        v[q] = keep + dpp_f64<CTRL>(send);
      }
    } else {
      v[0] += dpp_f64<CTRL>(v[0]);
    }
  }
}

template <int S, int B, int BIT, int NV>
__device__ __forceinline__ void group_rs_from(double (&v)[NV], int lane) {
  if constexpr (BIT >= 0) {
    constexpr int done = B - 1 - BIT;                       // halving steps so far
    constexpr int L = done < S ? (NV >> done) : 1;          // values left before this step
    rs_step<BIT, L, NV>(v, lane);
    group_rs_from<S, B, BIT - 1, NV>(v, lane);
  }
}

template <int S, int B>
__device__ __forceinline__ void group_reduce_scatter_d(double (&v)[1 << S], int lane) {
  static_assert(B >= 1 && B <= 6, "groups of 2 to 64 lanes");
  group_rs_from<S, B, B - 1, (1 << S)>(v, lane);
}

// One DPP halving step of wave_reduce_scatter_d: L values in, L / 2 out (or a plain sum of
// the last one).  The DPP pattern pairs each lane with a lane that differs from it in BIT.
template <int CTRL, int BIT, int L, int NV>
__device__ __forceinline__ void rs_step_dpp(double (&v)[NV], int lane) {
  if constexpr (L > 1) {
    const bool hi = (lane & BIT) != 0;
#pragma unroll
    for (int q = 0; q < L / 2; ++q) {
      const double keep = hi ? v[q + L / 2] : v[q];
      const double send = hi ? v[q] : v[q + L / 2];
      v[q] = keep + dpp_f64<CTRL>(send);
    }
  } else {
    v[0] += dpp_f64<CTRL>(v[0]);
  }
}

// Reduce-scatter of NV = 2^S (S <= 6) float64 values over the 64 lanes of a wave, on the
// vector unit.  Halving steps over lane bits 5, 4 (permlane swaps), 3, 2 (row and half-row
// mirrors), 1, 0 (quad permutations): at each, a lane keeps the half of its values selected
// by that bit and adds its partner's copy of the same half.  Once one value is left the
// remaining bits are summed outright.  On return v[0] of lane l holds the wave total of value
// l >> (6 - S).
template <int S>
__device__ __forceinline__ void wave_reduce_scatter_d(double (&v)[1 << S], int lane) {
  static_assert(S >= 0 && S <= 6, "at most 64 values");
  constexpr int NV = 1 << S;
  // bit 5
  if constexpr (S >= 1) {
#pragma unroll
    for (int q = 0; q < NV / 2; ++q) {
      swap32_f64(v[q], v[q + NV / 2]);
      v[q] += v[q + NV / 2];
    }
  } else {
    double w = v[0];
    swap32_f64(v[0], w);
    v[0] += w;
  }
  // bit 4
  if constexpr (S >= 2) {
#pragma unroll
    for (int q = 0; q < NV / 4; ++q) {
      swap16_f64(v[q], v[q + NV / 4]);
      v[q] += v[q + NV / 4];
    }
  } else {
    double w = v[0];
    swap16_f64(v[0], w);
    v[0] += w;
  }
  rs_step_dpp<kDppMirror, 8, (S >= 3 ? NV / 4 : 1)>(v, lane);
  rs_step_dpp<kDppHalfMirror, 4, (S >= 4 ? NV / 8 : 1)>(v, lane);
  rs_step_dpp<kDppXor2, 2, (S >= 5 ? NV / 16 : 1)>(v, lane);
  rs_step_dpp<kDppXor1, 1, (S >= 6 ? NV / 32 : 1)>(v, lane);
}

// (max, sum) merge across the 64 lanes of a wave: DPP inside each row of 16 lanes, then a
// lane swizzle across rows (xor 16) and a read of lane 32 for the last step.  The result is
// valid in lane 0.
__device__ __forceinline__ void wave_lse_merge(float& M, float& S) {
  float m2 = dpp_f32<kDppXor1>(M), s2 = dpp_f32<kDppXor1>(S);
  lse_merge(M, S, m2, s2);
  m2 = dpp_f32<kDppXor2>(M); s2 = dpp_f32<kDppXor2>(S);
  lse_merge(M, S, m2, s2);
  m2 = dpp_f32<kDppHalfMirror>(M); s2 = dpp_f32<kDppHalfMirror>(S);
  lse_merge(M, S, m2, s2);
  m2 = dpp_f32<kDppMirror>(M); s2 = dpp_f32<kDppMirror>(S);
  lse_merge(M, S, m2, s2);
  // xor 16 within each half-wave (ds_swizzle bit mode: and 0x1f, xor 0x10)
  m2 = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(M), 0x401F));
  s2 = __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(S), 0x401F));
  lse_merge(M, S, m2, s2);
  m2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(M), 32));
  s2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(S), 32));
  lse_merge(M, S, m2, s2);
}

// Block-wide sum of a double; every thread gets the result.  `scratch` holds >= nwaves
// doubles of shared memory.  Must be called by all threads of the block.
__device__ __forceinline__ double block_sum_d(double v, double* scratch) {
  v = wave_sum_d(v);
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < nw; ++w) t += scratch[w];
  __syncthreads();
  return t;
}

// Bound on the polls of a bounded wait (seconds of polling); after it the waiter raises the abort
// flag, which every other waiter checks, so a grid always drains.
constexpr uint32_t kSpinLimit = 1u << 22;

// ----------------------------------------------------------------------------------------
// Epoch-tagged exchange slots.
//
// A slot is one 64-bit word holding a float value in the low half and the iteration (epoch)
// that produced it in the high half, written with a single relaxed agent-scope atomic store.
// A consumer polls the slot with relaxed agent-scope atomic loads until the epoch it needs
// appears, so the word is its own ready flag: no counter barrier, no cache write-back or
// invalidate fences.  Per-location coherence of atomics guarantees the poll eventually sees
// the store; single-copy atomicity of the aligned 64-bit word guarantees value and epoch
// belong together.  Polls are bounded: a consumer that spins kSpinLimit times raises the
// abort flag, and every poller checks that flag, so a grid always drains.
// ----------------------------------------------------------------------------------------
__device__ __forceinline__ void slot_publish(uint64_t* slot, float v, uint32_t epoch) {
  const uint64_t w = ((uint64_t)epoch << 32) | (uint64_t)__float_as_uint(v);
  __hip_atomic_store(slot, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publication visible only through the L2 of the writer's XCD: a plain (workgroup-scope)
// store, which the write-through L1 forwards to that L2, where agent-scope loads from CUs of
// the same XCD find it.  Agent-scope stores are written through to memory as well and take
// about twice as long to reach a poller.  Only for grids whose workgroups have been checked
// to share one XCD (see xcc_id); across XCDs such a store stays in the writer's L2 and the
// bounded polls of the other side would time out.
__device__ __forceinline__ void slot_publish_local(uint64_t* slot, float v, uint32_t epoch) {
  const uint64_t w = ((uint64_t)epoch << 32) | (uint64_t)__float_as_uint(v);
  __hip_atomic_store(slot, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Index of the XCD (accelerator complex die) this wave runs on: hardware register XCC_ID,
// bits [3:0].
__device__ __forceinline__ uint32_t xcc_id() {
  return (uint32_t)__builtin_amdgcn_s_getreg((3 << 11) | 20) & 15u;
}

__device__ __forceinline__ uint64_t slot_load(uint64_t* slot) {
  return __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until `w` (already loaded from `slot`) carries `epoch`; returns false on abort.
// Polls are pipelined: DEPTH loads are in flight, a new one issued before the oldest is
// examined, so a poll leaves every 1/DEPTH of a round trip; SLEEP (units of 64 cycles) spaces
// them further.
template <int SLEEP = 2, int DEPTH = 2>
__device__ __forceinline__ bool slot_wait(uint64_t* slot, uint64_t& w, uint32_t epoch,
                                          uint32_t* abort_flag) {
  static_assert(DEPTH >= 2, "at least two polls in flight");
  if ((uint32_t)(w >> 32) == epoch) return true;
  uint32_t spins = 0;
  uint64_t q[DEPTH - 1];
#pragma unroll
  for (int k = 0; k < DEPTH - 1; ++k) q[k] = slot_load(slot);
  for (;;) {
    if constexpr (SLEEP > 0) __builtin_amdgcn_s_sleep(SLEEP);
    const uint64_t after = slot_load(slot);
    w = q[0];
    if ((uint32_t)(w >> 32) == epoch) return true;
#pragma unroll
    for (int k = 0; k + 1 < DEPTH - 1; ++k) q[k] = q[k + 1];
    q[DEPTH - 2] = after;
    if (++spins >= kSpinLimit) {
      __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    if ((spins & 63u) == 0 &&
        __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
      return false;
  }
}

// alpha * (2^d - 1), accurate also for tiny d (series below 2^-5, exp2 otherwise).
__device__ __forceinline__ float scaled_exp2m1(float alpha, float d) {
  const float u = d * kLn2;
  if (fabsf(d) < 0.03125f)
    return alpha * u * (1.0f + u * (0.5f + u * (0.16666667f + u * (0.041666668f + u * 0.008333334f))));
  return alpha * (exp2_fast(d) - 1.0f);
}

__device__ __forceinline__ float slot_value(uint64_t w) {
  return __uint_as_float((uint32_t)(w & 0xffffffffull));
}

// Stage the m slots of `src` carrying `epoch` into Vs (zero padding up to mp) and, when
// `extra` is non-null, the `nextra` slots of `extra` into xv.  Every thread issues all its
// loads first and then waits on the ones not yet current, so both sets cost one round trip.
// Returns false on abort.
template <int SLEEP = 2, int DEPTH = 2>
__device__ __forceinline__ bool stage_slots(uint64_t* src, int m, int mp, uint32_t epoch,
                                            float* Vs, uint64_t* extra, int nextra,
                                            uint32_t xepoch, float* xv, uint32_t* abort_flag,
                                            int* s_bad) {
  constexpr int kB = 2;
  bool ok = true;
  const int total = mp + nextra;
  for (int base = threadIdx.x; base < total; base += kB * (int)blockDim.x) {
    uint64_t w[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int j = base + u * (int)blockDim.x;
      w[u] = j < m ? slot_load(src + j)
                   : (j >= mp && j < total) ? slot_load(extra + (j - mp)) : 0ull;
    }
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int j = base + u * (int)blockDim.x;
      if (j < m) {
        if (ok) ok = slot_wait<SLEEP, DEPTH>(src + j, w[u], epoch, abort_flag);
        Vs[j] = slot_value(w[u]);
      } else if (j < mp) {
        Vs[j] = 0.0f;
      } else if (j < total) {
        if (ok) ok = slot_wait<SLEEP, DEPTH>(extra + (j - mp), w[u], xepoch, abort_flag);
        xv[j - mp] = slot_value(w[u]);
      }
    }
  }
  if (!ok) *s_bad = 1;
  __syncthreads();
  return *s_bad == 0;
}

// Zero `count` 32-bit words (control blocks) -- a kernel rather than a memset so that a
// captured graph holds no memset node.
__global__ void zero_words_kernel(uint32_t* p, int count);

}  // namespace csot
