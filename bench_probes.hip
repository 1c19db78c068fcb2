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
//   mfma    one launch per matrix instruction the library uses (FP32 16x16x4,
//           FP64 16x16x4, BF16 16x16x32), each issuing a known number of
//           wave-level MFMAs, to check the SQ_INSTS_VALU_MFMA_MOPS_* counters
//           (512 flops a count) and time the instruction's issue rate.
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

typedef float float4_v __attribute__((ext_vector_type(4)));
typedef double double4_v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_v __attribute__((ext_vector_type(8)));

// kMfmaChains independent accumulators per wave, kMfmaUnroll rounds per
// iteration: iters x kMfmaUnroll x kMfmaChains wave-level MFMAs per wave.
constexpr int kMfmaChains = 4;
constexpr int kMfmaUnroll = 8;

__global__ __launch_bounds__(256) void k_mfma_f32(float* out, int iters) {
  const float a = 1.0f + threadIdx.x * 1e-6f, b = 0.5f - threadIdx.x * 1e-6f;
  float4_v acc[kMfmaChains];
  for (int c = 0; c < kMfmaChains; ++c) acc[c] = float4_v{0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < kMfmaUnroll; ++r)
#pragma unroll
      for (int c = 0; c < kMfmaChains; ++c)
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
  }
  float t = 0.f;
  for (int c = 0; c < kMfmaChains; ++c) t += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_mfma_f64(float* out, int iters) {
  const double a = 1.0 + threadIdx.x * 1e-6, b = 0.5 - threadIdx.x * 1e-6;
  double4_v acc[kMfmaChains];
  for (int c = 0; c < kMfmaChains; ++c) acc[c] = double4_v{0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < kMfmaUnroll; ++r)
#pragma unroll
      for (int c = 0; c < kMfmaChains; ++c)
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double t = 0.0;
  for (int c = 0; c < kMfmaChains; ++c) t += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = float(t);
}

__global__ __launch_bounds__(256) void k_mfma_bf16(float* out, int iters) {
  bf16x8_v a, b;
  for (int q = 0; q < 8; ++q) {
    a[q] = static_cast<__bf16>(1.0f + (threadIdx.x + q) * 1e-3f);
    b[q] = static_cast<__bf16>(0.5f - (threadIdx.x + q) * 1e-3f);
  }
  float4_v acc[kMfmaChains];
  for (int c = 0; c < kMfmaChains; ++c) acc[c] = float4_v{0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < kMfmaUnroll; ++r)
#pragma unroll
      for (int c = 0; c < kMfmaChains; ++c)
        acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
  }
  float t = 0.f;
  for (int c = 0; c < kMfmaChains; ++c) t += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
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

// One launch of a matrix-instruction probe: 256 workgroups of 4 waves, each
// wave iters x kMfmaUnroll x kMfmaChains MFMAs of flops_each flops.
template <typename Kern>
void mfma_count(float* out, Kern kern, const char* name, const char* counter, int flops_each) {
  const int blocks = 256, iters = 2000;
  const double ms = time_ms([&] {
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, 0, out, iters);
  });
  if (ms < 0) return;
  // the probe launches twice (warm-up and timed): per launch
  const double insts = double(blocks) * 4 * iters * kMfmaUnroll * kMfmaChains;
  std::printf(
      "{\"probe\": \"mfma\", \"instruction\": \"%s\", \"counter\": \"%s\", "
      "\"wave_mfma_per_launch\": %.0f, \"flops_each\": %d, "
      "\"expected_counter_per_launch_at_512_flops\": %.0f, \"ms\": %.4f, "
      "\"tflops\": %.2f}\n",
      name, counter, insts, flops_each, insts * flops_each / 512.0, ms,
      insts * flops_each / (ms * 1e-3) / 1e12);
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
  if (all || !std::strcmp(mode, "mfma")) {
    mfma_count(out, k_mfma_f32, "v_mfma_f32_16x16x4_f32", "SQ_INSTS_VALU_MFMA_MOPS_F32",
               16 * 16 * 4 * 2);
    mfma_count(out, k_mfma_f64, "v_mfma_f64_16x16x4_f64", "SQ_INSTS_VALU_MFMA_MOPS_F64",
               16 * 16 * 4 * 2);
    mfma_count(out, k_mfma_bf16, "v_mfma_f32_16x16x32_bf16", "SQ_INSTS_VALU_MFMA_MOPS_BF16",
               16 * 16 * 32 * 2);
  }
  (void)hipFree(out);
  return 0;
}
