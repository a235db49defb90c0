// Measured MFMA throughput of the device: the ceiling that the product's
// roofline is compared against, next to the published dense peak.
#include <vector>

#include "kern.hpp"
#include "tns_internal.hpp"

namespace tns {

constexpr int PEAK_CHAINS = 8;  // independent accumulators per wave: the MFMA pipe never waits on a result
constexpr int PEAK_THREADS = 256;

// Each wave issues iters x PEAK_CHAINS independent MFMAs on register operands
// (accumulators pinned to registers, so that the loop is the MFMA sequence alone)
// and writes one value per lane, so that nothing is optimised away.
#define TNS_PEAK_LOOP(OP, CC)                                                                \
  for (int i = 0; i < iters; ++i) {                                                           \
    asm volatile(OP " %0, %1, %2, %0" : CC(c0) : "v"(a), "v"(b));                             \
    asm volatile(OP " %0, %1, %2, %0" : CC(c1) : "v"(a), "v"(b));                             \
    asm volatile(OP " %0, %1, %2, %0" : CC(c2) : "v"(a), "v"(b));                             \
    asm volatile(OP " %0, %1, %2, %0" : CC(c3) : "v"(a), "v"(b));                             \
    asm volatile(OP " %0, %1, %2, %0" : CC(c4) : "v"(a), "v"(b));                             \
    asm volatile(OP " %0, %1, %2, %0" : CC(c5) : "v"(a), "v"(b));                             \
    asm volatile(OP " %0, %1, %2, %0" : CC(c6) : "v"(a), "v"(b));                             \
    asm volatile(OP " %0, %1, %2, %0" : CC(c7) : "v"(a), "v"(b));                             \
  }
static_assert(PEAK_CHAINS == 8, "the peak loop runs eight accumulators");

template <class A4>
__device__ inline float peak_sum(A4 c0, A4 c1, A4 c2, A4 c3, A4 c4, A4 c5, A4 c6, A4 c7) {
  const A4 t = ((c0 + c1) + (c2 + c3)) + ((c4 + c5) + (c6 + c7));
  return (float)((t[0] + t[1]) + (t[2] + t[3]));
}

template <int P>
__global__ __launch_bounds__(PEAK_THREADS) void k_mfma_peak(int iters, float *out) {
  const int lane = threadIdx.x & 63;
  float s;
  if constexpr (P == TNS_F64) {
    const double a = 1e-3 * (lane + 1), b = 1e-3 * (lane + 2);
    d4 c0 = vzero<d4>(), c1 = c0, c2 = c0, c3 = c0, c4 = c0, c5 = c0, c6 = c0, c7 = c0;
    TNS_PEAK_LOOP("v_mfma_f64_16x16x4_f64", "+v")
    s = peak_sum(c0, c1, c2, c3, c4, c5, c6, c7);
  } else if constexpr (P == TNS_F32) {
    const float a = 1e-3f * (lane + 1), b = 1e-3f * (lane + 2);
    f4 c0 = vzero<f4>(), c1 = c0, c2 = c0, c3 = c0, c4 = c0, c5 = c0, c6 = c0, c7 = c0;
    TNS_PEAK_LOOP("v_mfma_f32_16x16x4_f32", "+a")
    s = peak_sum(c0, c1, c2, c3, c4, c5, c6, c7);
  } else {
    u16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[e] = f32_to_bf16_rne(1e-3f * (lane + e));
      b[e] = f32_to_bf16_rne(1e-3f * (lane - e));
    }
    f4 c0 = vzero<f4>(), c1 = c0, c2 = c0, c3 = c0, c4 = c0, c5 = c0, c6 = c0, c7 = c0;
    TNS_PEAK_LOOP("v_mfma_f32_16x16x32_bf16", "+a")
    s = peak_sum(c0, c1, c2, c3, c4, c5, c6, c7);
  }
  out[(int64_t)blockIdx.x * PEAK_THREADS + threadIdx.x] = s;
}

// Flops of one MFMA instruction of the precision's product.
static double mfma_flops(tns_prec p) {
  return p == TNS_BF16X3 ? 2.0 * 16 * 16 * 32 : 2.0 * 16 * 16 * 4;
}

}  // namespace tns

using namespace tns;

extern "C" size_t tns_mfma_peak_workspace_bytes(void) {
  int dev = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu <= 0)
    return 0;
  return (size_t)n_cu * 8 * PEAK_THREADS * sizeof(float);
}

extern "C" tns_status tns_mfma_peak(tns_prec prec, int iters, void *ws, size_t ws_bytes, double *tflops,
                                    hipStream_t st) {
  if (!tflops || !ws || iters <= 0) return TNS_ERR_ARG;
  if (prec != TNS_F64 && prec != TNS_F32 && prec != TNS_BF16X3) return TNS_ERR_ARG;
  const size_t need = tns_mfma_peak_workspace_bytes();
  if (need == 0) return TNS_ERR_HIP;
  if (ws_bytes < need) return TNS_ERR_WORKSPACE;
  const int blocks = (int)(need / (PEAK_THREADS * sizeof(float)));  // 8 workgroups (32 waves) per CU
  float *out = reinterpret_cast<float *>(ws);
  auto launch = [&]() {
    if (prec == TNS_F64) hipLaunchKernelGGL(k_mfma_peak<TNS_F64>, dim3(blocks), dim3(PEAK_THREADS), 0, st, iters, out);
    else if (prec == TNS_F32) hipLaunchKernelGGL(k_mfma_peak<TNS_F32>, dim3(blocks), dim3(PEAK_THREADS), 0, st, iters, out);
    else hipLaunchKernelGGL(k_mfma_peak<TNS_BF16X3>, dim3(blocks), dim3(PEAK_THREADS), 0, st, iters, out);
  };
  hipEvent_t e0, e1;
  TNS_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return TNS_ERR_HIP;
  }
  std::vector<float> t;
  tns_status s = TNS_OK;
  launch();  // warm-up
  for (int r = 0; r < 5 && s == TNS_OK; ++r) {
    float ms = 0.f;
    if (hipEventRecord(e0, st) != hipSuccess) { s = TNS_ERR_HIP; break; }
    launch();
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess || hipGetLastError() != hipSuccess) {
      s = TNS_ERR_HIP;
      break;
    }
    t.push_back(ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != TNS_OK) return s;
  float best = t[0];
  for (float x : t) best = x < best ? x : best;
  const double flops = (double)blocks * (PEAK_THREADS / 64) * (double)iters * PEAK_CHAINS * mfma_flops(prec);
  *tflops = flops / (best * 1e-3) / 1e12;
  return TNS_OK;
}
