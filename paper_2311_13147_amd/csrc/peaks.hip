// Micro-benchmarks of the current device: the issue rates and latencies the roofline figures
// of the solvers are quoted against (not a step of the method).
//
//   fp32 FMA    v_fma_f32 on 8 independent chains per lane (non-packed; this build emits no
//               packed FP32 instructions)
//   fp64 FMA    v_fma_f64, likewise
//   exp2        v_exp_f32 on 8 independent chains, y <- 2^-y (stays in [1/2, 1])
//   entry mix   the full-size Sinkhorn inner step per (I, J) entry on pre-scaled coordinates
//               in registers: 2 subtractions, 2 FMAs, one exp2 and the accumulation -- the
//               instruction mix whose issue rate bounds the full-size solver
//   fp64 MFMA   v_mfma_f64_16x16x4f64 (16 x 4 by 4 x 16, 1024 multiply-adds) on 8 independent
//               accumulators per wave -- the matrix cores the batched gradients run on
//   copy        float4 device-to-device copy of a buffer much larger than the caches
//   slot hop    one-way latency of an epoch-tagged slot (common.hpp) between two workgroups:
//               on one XCD with XCD-local publication (the reduced solver's exchange) and
//               across XCDs with device-scope publication
// Rates count lane operations (a wave64 instruction is 64).
#include <cmath>

#include "common.hpp"
#include "launch.hpp"

namespace csot {

constexpr int kPeakThreads = 256;
constexpr int kPeakChains = 8;

__global__ void __launch_bounds__(kPeakThreads) peak_fma32_kernel(float* out, int iters, float a,
                                                                  float b) {
  float v[kPeakChains];
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) v[c] = (float)(threadIdx.x & 7) * 1e-3f + (float)c;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int c = 0; c < kPeakChains; ++c) v[c] = fmaf(v[c], a, b);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) s += v[c];
  if (s == -1.0f) out[blockIdx.x] = s;  // never true: keeps the chains live
}

__global__ void __launch_bounds__(kPeakThreads) peak_fma64_kernel(double* out, int iters, double a,
                                                                  double b) {
  double v[kPeakChains];
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) v[c] = (double)(threadIdx.x & 7) * 1e-3 + (double)c;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int c = 0; c < kPeakChains; ++c) v[c] = fma(v[c], a, b);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) s += v[c];
  if (s == -1.0) out[blockIdx.x] = s;
}

typedef double v4d_peak __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kPeakThreads) peak_mfma64_kernel(double* out, int iters) {
  v4d_peak acc[kPeakChains];
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) acc[c] = v4d_peak{0.0, 0.0, 0.0, 0.0};
  const double a = 1.0 + 1e-3 * (threadIdx.x & 15), b = 1e-7 * (1 + (threadIdx.x >> 4));
  for (int it = 0; it < iters; ++it) {
    // 16 rounds per loop trip: the compiler moves the accumulators between register files once
    // per trip (128 moves against 128 MFMAs of 64 cycles each), so that they do not count
#pragma unroll
    for (int u = 0; u < 16; ++u)
#pragma unroll
      for (int c = 0; c < kPeakChains; ++c)
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) s += (acc[c][0] + acc[c][1]) + (acc[c][2] + acc[c][3]);
  if (s == -1.0) out[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kPeakThreads) peak_exp2_kernel(float* out, int iters) {
  float v[kPeakChains];
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) v[c] = 0.5f + 0.01f * (float)c + 1e-4f * (threadIdx.x & 7);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int c = 0; c < kPeakChains; ++c) v[c] = exp2_fast(-v[c]);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) s += v[c];
  if (s == -1.0f) out[blockIdx.x] = s;
}

// 4 rows (own points) against 8 partner columns per step: 32 entries, each as the full-size
// solver evaluates it on coordinates pre-scaled by sqrt(log2(e)/eps) with the shift folded
// into the staged potential: z = G_J - (x_I0 - y_J0)^2 - (x_I1 - y_J1)^2 as 2 subtractions and
// 2 FMAs, then exp2 and the accumulation.  The partner columns move once per step (2 adds per
// column: a quarter of an instruction per entry on top).
__global__ void __launch_bounds__(kPeakThreads) peak_mix_kernel(float* out, int iters) {
  float xi[4][2], acc[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    xi[r][0] = 0.1f * r + 1e-3f * (threadIdx.x & 15);
    xi[r][1] = 0.2f - 0.05f * r;
    acc[r] = 0.0f;
  }
  float yj[8][2], gj[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    yj[c][0] = 0.05f * c;
    yj[c][1] = -0.03f * c;
    gj[c] = -0.5f * c;
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float dx = xi[r][0] - yj[c][0];
        const float dy = xi[r][1] - yj[c][1];
        const float z = fmaf(-dy, dy, fmaf(-dx, dx, gj[c]));
        acc[r] += exp2_fast(z);
      }
      yj[c][0] += 1e-7f;
      yj[c][1] -= 1e-7f;
    }
  }
  float s = acc[0] + acc[1] + acc[2] + acc[3];
  if (s == -1.0f) out[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kPeakThreads) peak_copy_kernel(const float4* __restrict__ src,
                                                                 float4* __restrict__ dst,
                                                                 int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
    dst[i] = src[i];
}

// Ping-pong between block 0 and block `partner` (the other blocks exit at once): block 0
// publishes epoch e in slot A, the partner waits for it and publishes e in slot B, block 0
// waits for that, for e = 1 .. hops.  `local` asks for XCD-local publication, which is used
// only when both blocks report the same XCD (checked first through device-scope slots); the
// outcome is written to res[0] (1: local publication used).  Bounded waits: on a timeout the
// abort flag ends both loops.
__global__ void __launch_bounds__(64) peak_hop_kernel(uint64_t* slots, uint32_t* abort_flag,
                                                      int partner, int hops, int local,
                                                      double* res) {
  const int b = blockIdx.x;
  if ((b != 0 && b != partner) || threadIdx.x != 0) return;
  const bool me0 = b == 0;
  uint64_t* xid = slots + 2;  // [2] XCD ids (epoch 1)
  slot_publish(xid + (me0 ? 0 : 1), __uint_as_float(xcc_id()), 1u);
  uint64_t w = slot_load(xid + (me0 ? 1 : 0));
  if (!slot_wait(xid + (me0 ? 1 : 0), w, 1u, abort_flag)) return;
  const bool same = __float_as_uint(slot_value(w)) == xcc_id();
  const bool loc = local && same;
  if (me0) res[0] = loc ? 1.0 : 0.0;
  uint64_t* mine = slots + (me0 ? 0 : 1);
  uint64_t* theirs = slots + (me0 ? 1 : 0);
  for (int e = 1; e <= hops; ++e) {
    const uint32_t ep = (uint32_t)e + 1u;  // epochs 2.. (1 is the id exchange)
    if (me0) {
      if (loc) slot_publish_local(mine, 0.0f, ep); else slot_publish(mine, 0.0f, ep);
      uint64_t v = slot_load(theirs);
      if (!slot_wait(theirs, v, ep, abort_flag)) return;
    } else {
      uint64_t v = slot_load(theirs);
      if (!slot_wait(theirs, v, ep, abort_flag)) return;
      if (loc) slot_publish_local(mine, 0.0f, ep); else slot_publish(mine, 0.0f, ep);
    }
  }
}

namespace {

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  ~EventPair() {
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
  }
};

// Time `launch` (called twice: warm-up, then timed) in seconds.
template <class F>
hipError_t timed(F launch, hipStream_t s, double* sec) {
  EventPair ev;
  hipError_t e;
  if ((e = hipEventCreate(&ev.a)) != hipSuccess || (e = hipEventCreate(&ev.b)) != hipSuccess)
    return e;
  launch();
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipEventRecord(ev.a, s)) != hipSuccess) return e;
  launch();
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipEventRecord(ev.b, s)) != hipSuccess) return e;
  if ((e = hipEventSynchronize(ev.b)) != hipSuccess) return e;
  float ms = 0.0f;
  if ((e = hipEventElapsedTime(&ms, ev.a, ev.b)) != hipSuccess) return e;
  *sec = ms * 1e-3;
  return hipSuccess;
}

}  // namespace

size_t peaks_scratch_bytes() { return kPeaksCopyBytes * 2 + 4096; }

hipError_t measure_peaks(double* out, void* scratch, hipStream_t s) {
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  char* base = static_cast<char*>(scratch);
  float* sink = reinterpret_cast<float*>(base);                // [1024] never written
  uint64_t* slots = reinterpret_cast<uint64_t*>(base + 2048);  // [4]
  uint32_t* abort_flag = reinterpret_cast<uint32_t*>(base + 2048 + 64);
  double* res = reinterpret_cast<double*>(base + 2048 + 128);
  float4* src = reinterpret_cast<float4*>(base + 4096);
  float4* dst = reinterpret_cast<float4*>(base + 4096 + kPeaksCopyBytes);

  const int blocks = cus * 8;  // 8 workgroups of 4 waves per CU: 8 waves per SIMD
  const double lanes = (double)blocks * kPeakThreads;
  double t = 0.0;
  // fp32 FMA
  const int it32 = 4096;
  if ((e = timed([&] { hipLaunchKernelGGL(peak_fma32_kernel, dim3(blocks), dim3(kPeakThreads), 0, s,
                                          sink, it32, 0.9999999f, 1e-7f); },
                 s, &t)) != hipSuccess)
    return e;
  out[0] = lanes * it32 * 8 * kPeakChains / t;
  // fp64 FMA
  if ((e = timed([&] { hipLaunchKernelGGL(peak_fma64_kernel, dim3(blocks), dim3(kPeakThreads), 0, s,
                                          reinterpret_cast<double*>(sink), it32, 0.9999999, 1e-7); },
                 s, &t)) != hipSuccess)
    return e;
  out[1] = lanes * it32 * 8 * kPeakChains / t;
  // exp2
  const int itx = 1024;
  if ((e = timed([&] { hipLaunchKernelGGL(peak_exp2_kernel, dim3(blocks), dim3(kPeakThreads), 0, s,
                                          sink, itx); },
                 s, &t)) != hipSuccess)
    return e;
  out[2] = lanes * itx * 8 * kPeakChains / t;
  // full-size entry mix: 32 entries per step
  const int itm = 1024;
  if ((e = timed([&] { hipLaunchKernelGGL(peak_mix_kernel, dim3(blocks), dim3(kPeakThreads), 0, s,
                                          sink, itm); },
                 s, &t)) != hipSuccess)
    return e;
  out[3] = lanes * itm * 32 / t;
  // copy (read + write bytes)
  const int64_t n4 = (int64_t)(kPeaksCopyBytes / sizeof(float4));
  if ((e = timed([&] { hipLaunchKernelGGL(peak_copy_kernel, dim3(cus * 16), dim3(kPeakThreads), 0, s,
                                          src, dst, n4); },
                 s, &t)) != hipSuccess)
    return e;
  out[4] = 2.0 * (double)kPeaksCopyBytes / t;
  // slot hops: block 8 shares block 0's XCD when blocks are dealt round-robin to 8 XCDs;
  // block 1 is on the next XCD
  const int hops = 20000;
  for (int v = 0; v < 2; ++v) {
    const int partner = v == 0 ? 8 : 1;
    double tt = 0.0;
    auto run = [&] {
      launch_zero_words(reinterpret_cast<uint32_t*>(slots), 32, s);
      hipLaunchKernelGGL(peak_hop_kernel, dim3(partner + 1), dim3(64), 0, s, slots, abort_flag,
                         partner, hops, v == 0 ? 1 : 0, res);
    };
    if ((e = timed(run, s, &tt)) != hipSuccess) return e;
    uint32_t ab = 0;
    double used_local = 0.0;
    if ((e = hipMemcpy(&ab, abort_flag, 4, hipMemcpyDeviceToHost)) != hipSuccess) return e;
    if ((e = hipMemcpy(&used_local, res, 8, hipMemcpyDeviceToHost)) != hipSuccess) return e;
    // one round trip is two one-way hops
    out[5 + v] = ab ? NAN : tt / (2.0 * hops);
    if (v == 0) out[7] = used_local;
  }
  // fp64 matrix cores: 1024 multiply-adds per wave instruction
  const int itf = 256;
  if ((e = timed([&] { hipLaunchKernelGGL(peak_mfma64_kernel, dim3(blocks), dim3(kPeakThreads), 0,
                                          s, reinterpret_cast<double*>(sink), itf); },
                 s, &t)) != hipSuccess)
    return e;
  out[8] = (double)blocks * (kPeakThreads / kWave) * itf * 16 * kPeakChains * 1024.0 / t;
  return hipSuccess;
}

}  // namespace csot
