// Issue-rate probes of the vector operations the depth recursion is built
// from: FP32 FMA (non-packed: packed FP32 is disabled at compile time),
// FP64 FMA, the FP32 exponential (v_exp_f32) and reciprocal (v_rcp_f32).
// They supply the denominators of the recursion's VALU roofline: issue
// slots per second, and what a transcendental costs in FMA slots.
// Measurement only; nothing of the method runs here.
#include <hip/hip_runtime.h>

#include "nlte_internal.h"

nlte_status set_err(nlte_status st, const char* fmt, ...);

#define HIP_TRY(x)                                                                     \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      return set_err(NLTE_E_DEVICE, "%s failed: %s", #x, hipGetErrorString(e_));       \
  } while (0)

namespace {

constexpr int kChains = 8;          // independent dependency chains per lane
constexpr int kProbeThreads = 256;
constexpr int kProbeUnroll = 4;     // iterations per loop trip

// Every lane runs kChains independent chains of `iters` operations of one
// kind, so that with a full device the issue rate, not the latency of a
// chain, sets the time.  The chains stay finite: FMAs contract towards a
// fixed point, exp2(-x) maps (0, 1] into [1/2, 1), 1/x alternates between
// two values.  The sum is written out so that nothing is optimised away.
template <int OP>
__global__ __launch_bounds__(kProbeThreads) void k_issue_probe(double* out, int iters) {
  const int tid = blockIdx.x * kProbeThreads + threadIdx.x;
  if constexpr (OP == NLTE_PROBE_FMA_F64) {
    double v[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) v[i] = 1.0 + 1e-3 * (tid & 7) + 1e-4 * i;
    for (int it = 0; it < iters; it += kProbeUnroll)
#pragma unroll
      for (int u = 0; u < kProbeUnroll; ++u)
#pragma unroll
        for (int i = 0; i < kChains; ++i) v[i] = __builtin_fma(v[i], 0.999999, 1e-7);
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += v[i];
    out[tid] = s;
  } else {
    float v[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) v[i] = 0.5f + 1e-3f * (tid & 7) + 1e-2f * i;
    for (int it = 0; it < iters; it += kProbeUnroll)
#pragma unroll
      for (int u = 0; u < kProbeUnroll; ++u)
#pragma unroll
        for (int i = 0; i < kChains; ++i) {
          if constexpr (OP == NLTE_PROBE_FMA_F32)
            v[i] = __builtin_fmaf(v[i], 0.999999f, 1e-7f);
          else if constexpr (OP == NLTE_PROBE_EXP_F32)
            v[i] = __builtin_amdgcn_exp2f(-v[i]);
          else
            v[i] = __builtin_amdgcn_rcpf(v[i]);
        }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += v[i];
    out[tid] = (double)s;
  }
}

template <int OP>
hipError_t launch_probe(int blocks, double* out, int iters, hipStream_t s) {
  k_issue_probe<OP><<<blocks, kProbeThreads, 0, s>>>(out, iters);
  return hipGetLastError();
}

hipError_t launch_op(int op, int blocks, double* out, int iters, hipStream_t s) {
  switch (op) {
    case NLTE_PROBE_FMA_F32: return launch_probe<NLTE_PROBE_FMA_F32>(blocks, out, iters, s);
    case NLTE_PROBE_FMA_F64: return launch_probe<NLTE_PROBE_FMA_F64>(blocks, out, iters, s);
    case NLTE_PROBE_EXP_F32: return launch_probe<NLTE_PROBE_EXP_F32>(blocks, out, iters, s);
    default: return launch_probe<NLTE_PROBE_RCP_F32>(blocks, out, iters, s);
  }
}

}  // namespace

extern "C" nlte_status nlte_issue_rate(nlte_ctx* ctx, int32_t op, int32_t iters,
                                       double* lane_ops_per_s) {
  if (!ctx || !lane_ops_per_s) return set_err(NLTE_E_INVALID, "NULL argument");
  if (op < NLTE_PROBE_FMA_F32 || op > NLTE_PROBE_RCP_F32)
    return set_err(NLTE_E_INVALID, "unknown probe operation %d", op);
  if (iters < kProbeUnroll || iters > (1 << 24) || iters % kProbeUnroll)
    return set_err(NLTE_E_INVALID, "iters = %d: a multiple of %d in [%d, 2^24]", iters,
                   kProbeUnroll, kProbeUnroll);
  HIP_TRY(hipSetDevice(ctx->device));
  int cus = 0;
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
  // eight 256-thread blocks per CU: 32 waves, the most a CU holds
  const int blocks = 8 * (cus > 0 ? cus : 1);
  hipStream_t s = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  double* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc((void**)&out, (size_t)blocks * kProbeThreads * sizeof(double));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = launch_op(op, blocks, out, iters, s);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  if (e == hipSuccess) e = launch_op(op, blocks, out, iters, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e1) (void)hipEventDestroy(e1);
  if (e0) (void)hipEventDestroy(e0);
  if (out) (void)hipFree(out);
  (void)hipStreamDestroy(s);
  if (e != hipSuccess) return set_err(NLTE_E_DEVICE, "issue-rate probe: %s", hipGetErrorString(e));
  if (!(ms > 0.0f)) return set_err(NLTE_E_DEVICE, "issue-rate probe: no elapsed time");
  *lane_ops_per_s = (double)blocks * kProbeThreads * (double)iters * kChains / (ms * 1e-3);
  return NLTE_OK;
}
