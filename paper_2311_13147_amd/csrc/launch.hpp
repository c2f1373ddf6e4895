// Host-side launchers of the csot kernels (internal; the public surface is include/csot.h).
// Every launcher enqueues on `stream` and returns the HIP status of the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "csot.h"

namespace csot {

// Geometry of one problem as the kernels see it.
struct Geom {
  int n, K, m, dim;
  const float* x;
  const float* y;
  const float* C;
  int64_t ldc;
  const float* a;
  const float* b;
  double eps;
};

// ---- lot.hip -----------------------------------------------------------------------------
hipError_t launch_lot_fold(const Geom& g, float* G, int32_t* kmin, float* alpha, float* beta,
                           hipStream_t s);
hipError_t launch_lot_expand(int m, int K, const float* S, const int32_t* kmin, float* T,
                             int64_t ldt, hipStream_t s);

// ---- srot.hip ----------------------------------------------------------------------------
size_t srot_ws_bytes(const Geom& g);
bool srot_supported(const Geom& g);
hipError_t run_srot(const Geom& g, double lam, double tol, int max_iter, int warm, float* w,
                    float* z, void* ws, double* res, hipStream_t s);

// ---- peaks.hip ---------------------------------------------------------------------------
constexpr size_t kPeaksCopyBytes = 256ull << 20;  // copy benchmark: source and destination each
size_t peaks_scratch_bytes();
hipError_t measure_peaks(double* out, void* scratch, hipStream_t s);

// ---- fold.hip ----------------------------------------------------------------------------
hipError_t launch_fold(const Geom& g, bool fp64, float* logK, float* alpha, float* beta,
                       hipStream_t s);
hipError_t launch_symmetrize(const Geom& g, float* Csym, int64_t ldcs, hipStream_t s);
hipError_t launch_zero_words(uint32_t* p, int count, hipStream_t s);

// ---- reduced.hip -------------------------------------------------------------------------
struct ReducedPlan {
  int W;        // cooperating workgroups
  int stride;   // launched blocks per workgroup (8 keeps the workgroups on one XCD)
  int R;        // rows (and columns) per workgroup
  int threads;  // threads per workgroup
  size_t lds;   // dynamic LDS bytes
  int gslab = 0;  // 1: logK slabs read from padded copies in the workspace (large m)
};
bool plan_reduced(int m, int workgroups_hint, ReducedPlan* plan);
// Bytes of the fixed device scratch behind ot_sinkhorn_reduced_noalloc (OT_REDUCED_SCRATCH_BYTES).
constexpr size_t kReducedScratchBytes = OT_REDUCED_SCRATCH_BYTES;
// Device address of that scratch on the current device (looked up once per device).
hipError_t reduced_scratch(void** ptr);
size_t reduced_ws_bytes(int m, const ReducedPlan& p);
hipError_t launch_sinkhorn_reduced(int m, int K, double eps, const float* logK,
                                   const float* alpha, const float* beta, float* f, float* g,
                                   double tol, int max_iter, int warm, double* dstats,
                                   void* ws, const ReducedPlan& p, hipStream_t s,
                                   hipEvent_t* events = nullptr);

// ---- full.hip ----------------------------------------------------------------------------
struct FullPlan {
  int W;
  int R;
  int P;  // row blocks of R rows per workgroup
  int threads;
  size_t lds;
};
bool plan_full(const Geom& g, int workgroups_hint, FullPlan* plan);
size_t full_ws_bytes(const Geom& g, const FullPlan& p);
hipError_t launch_sinkhorn_full(const Geom& g, float* f, float* gpot, double tol, int max_iter,
                                int warm, double* dstats, void* ws, const FullPlan& p,
                                hipStream_t s, hipEvent_t* events = nullptr);

// ---- expand.hip --------------------------------------------------------------------------
hipError_t launch_expand(const Geom& g, const float* f, const float* gp, float* T, int64_t ldt,
                         hipStream_t s);

// ---- costgrad.hip ------------------------------------------------------------------------
size_t costgrad_ws_bytes(const Geom& g);
hipError_t launch_check(const Geom& g, int reduced, const float* logK, const float* f,
                        const float* gp, const float* ra, const float* rb, double* sums,
                        double* dstats, hipStream_t s);
hipError_t launch_cost_and_grad(const Geom& g, const float* f, const float* gp, int reduced,
                                double* out, float* dC, int64_t lddc, float* dx, float* dy,
                                float* da, float* db, void* ws, hipStream_t s);

// ---- batched.hip -------------------------------------------------------------------------
size_t batched_plan_len(int count);
int batched_plan(const ot_batch_desc* host_descs, int count, int32_t* plan);
size_t batched_ws_bytes(int count);
hipError_t launch_batched(const ot_batch_desc* descs, int count, const int32_t* dplan,
                          const int32_t* hplan, double tol, int max_iter, int fold_fp64,
                          int warm, void* ws, hipStream_t s, hipEvent_t* events = nullptr);

}  // namespace csot
