// Issue-rate and counter-calibration probes for the pair kernels (built and
// run by `python bench.py --probes`; measurement code, not part of the
// library).
//
//   fma     independent unpacked FP32 FMAs (K accumulator chains per lane),
//           all operands in vector registers, or one multiplicand in a scalar
//           register, at 1 to 8 waves per SIMD (occupancy set through LDS);
//           reports cycles per wave-level FMA per SIMD at 2.4 GHz.
//   accum   the pair kernel's spin accumulation alone (SpinChunk::add, one
//           synthetic unit vector per lane per step) at 3 and 4 waves per SIMD.
//   count   one launch that issues exactly 2^20 wave-level FP32 FMAs, to check
//           what SQ_INSTS_VALU_FMA_F32 reads under rocprofv3.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>

#include "paper_1709_00086_amd/csrc/monomials.h"

using namespace g3;

namespace {

constexpr double kClock = 2.4e9;
constexpr int kSimds = 1024;  // 256 compute units x 4 SIMDs

template <int K, bool SCALAR_B>
__global__ __launch_bounds__(256) void k_fma(float* out, int iters, float a0, float b0) {
  const float a = SCALAR_B ? a0 : a0 + threadIdx.x * 1e-9f;
  const float b = b0 + threadIdx.x * 1e-9f;
  float acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = threadIdx.x * 1e-3f + k;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
#pragma unroll
      for (int k = 0; k < K; ++k) acc[k] = __builtin_fmaf(acc[k], a, b);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < K; ++k) s += acc[k];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <class Acc>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_accum(
    float* out, int iters, float c, float s) {
  Acc a;
  a.zero();
  float x = 0.6f + threadIdx.x * 1e-4f, y = 0.48f, z = 0.64f;
  const float w = 1.0f + threadIdx.x * 1e-5f;
  for (int it = 0; it < iters; ++it) {
    const float nx = fma_r(x, c, -(y * s)), ny = fma_r(x, s, y * c);
    x = nx;
    y = ny;
    a.add(x, y, z, w);
  }
  float t = 0.f;
#pragma unroll
  for (int i = 0; i < Acc::NT; ++i) t += a.acc[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

bool check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    std::printf("{\"error\": \"%s: %s\"}\n", what, hipGetErrorString(e));
    return false;
  }
  return true;
}

// Time the second of two launches (the first warms up).
template <typename Launch>
double time_ms(Launch&& launch) {
  hipEvent_t e0, e1;
  if (!check(hipEventCreate(&e0), "event") || !check(hipEventCreate(&e1), "event")) return -1;
  launch();
  if (!check(hipDeviceSynchronize(), "warm-up launch")) return -1;
  (void)hipEventRecord(e0);
  launch();
  (void)hipEventRecord(e1);
  if (!check(hipEventSynchronize(e1), "timed launch")) return -1;
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

template <int K, bool SCALAR_B>
void fma_rate(float* out, int waves_per_simd) {
  // one workgroup of 4 waves puts one wave on each SIMD of a compute unit;
  // the dynamic LDS share leaves room for waves_per_simd workgroups per unit
  const int blocks = 256 * waves_per_simd;
  const int lds = (160 * 1024) / waves_per_simd - 1024;
  const int iters = 1000;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_fma<K, SCALAR_B>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  const double ms = time_ms([&] {
    hipLaunchKernelGGL((k_fma<K, SCALAR_B>), dim3(blocks), dim3(256), lds, 0, out, iters,
                       0.999f, 1e-3f);
  });
  if (ms < 0) return;
  const double insts = double(blocks) * 4 * iters * 16 * K;  // wave-level FMAs
  std::printf(
      "{\"probe\": \"fma\", \"operands\": \"%s\", \"chains\": %d, \"waves_per_simd\": %d, "
      "\"ms\": %.4f, \"tflops\": %.2f, \"cycles_per_wave_fma\": %.3f}\n",
      SCALAR_B ? "one scalar multiplicand" : "vector registers", K, waves_per_simd, ms,
      insts * 128 / (ms * 1e-3) / 1e12, ms * 1e-3 * kClock / (insts / kSimds));
}

template <class Acc>
void accum_rate(float* out, const char* name, int waves_per_simd, int valu_per_step) {
  const int blocks = 256 * waves_per_simd, iters = 20000;
  const double ms = time_ms([&] {
    hipLaunchKernelGGL((k_accum<Acc>), dim3(blocks), dim3(256), 0, 0, out, iters, 0.9999f,
                       0.0141f);
  });
  if (ms < 0) return;
  const double steps = double(blocks) * 4 * iters;  // wave-level steps
  const double cyc = ms * 1e-3 * kClock / (steps / kSimds);
  std::printf(
      "{\"probe\": \"accum\", \"basis\": \"%s\", \"waves_per_simd\": %d, \"ms\": %.4f, "
      "\"cycles_per_wave_step\": %.1f, \"valu_per_step\": %d, \"cycles_per_valu\": %.3f}\n",
      name, waves_per_simd, ms, cyc, valu_per_step, cyc / valu_per_step);
}

}  // namespace

int main(int argc, char** argv) {
  const char* mode = argc > 1 ? argv[1] : "all";
  const bool all = std::strcmp(mode, "all") == 0;
  float* out = nullptr;
  if (!check(hipMalloc(&out, size_t(256) * 8 * 256 * sizeof(float)), "hipMalloc")) return 1;
  if (all || !std::strcmp(mode, "fma")) {
    for (int w : {1, 2, 3, 4, 8}) fma_rate<16, false>(out, w);
    for (int w : {3, 4, 8}) fma_rate<16, true>(out, w);
  }
  if (all || !std::strcmp(mode, "accum")) {
    // 164 VALU instructions per step: the accumulation's 159 and the
    // synthetic vector's 5 (counted in the compiled loop)
    for (int w : {3, 4}) accum_rate<SpinChunk<float, 0, kDeg>>(out, "spin", w, 164);
  }
  if (all || !std::strcmp(mode, "count")) {
    // 1024 waves x (4 iterations x 256 FMAs in the loop + 18 outside it: the
    // 16 initial values and the two per-lane operands, as compiled)
    hipLaunchKernelGGL((k_fma<16, false>), dim3(256), dim3(256), 0, 0, out, 4, 0.999f, 1e-3f);
    if (check(hipDeviceSynchronize(), "count launch"))
      std::printf("{\"probe\": \"count\", \"expected_wave_fma_f32\": %d}\n",
                  256 * 4 * (4 * 256 + 18));
  }
  (void)hipFree(out);
  return 0;
}
