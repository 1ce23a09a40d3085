// Calibration kernels: the rates this device reaches on the instruction
// types the detector is built from, measured rather than taken from the
// datasheet, so that roofline fractions can be stated against both.
//   kind 0: float32 FMA on the vector ALUs (eight independent chains per lane)
//   kind 1: v_mfma_f32_16x16x16_bf16 (four independent accumulator chains)
//   kind 2: v_mfma_f32_16x16x4_f32 (four independent accumulator chains)
// Each launch runs 1,024 workgroups of 256 threads (four waves per SIMD on
// 256 CUs); every lane stores one float so the work cannot be dropped.
#include "taser_internal.h"

namespace taser {
namespace {

constexpr int kCalibBlocks = 1024;
constexpr int kCalibThreads = 256;

__global__ __launch_bounds__(kCalibThreads) void calib_fma(int iters, float* __restrict__ out) {
  const int t = blockIdx.x * kCalibThreads + threadIdx.x;
  float a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = 1.f + 1e-3f * (float)((t + k) & 15);
  const float m = 0.9999f, c = 1e-4f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int k = 0; k < 8; ++k) a[k] = fmaf(a[k], m, c);
  }
  out[t] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kCalibThreads) void calib_mfma_bf16(int iters, float* __restrict__ out) {
  const int t = blockIdx.x * kCalibThreads + threadIdx.x;
  const short one = 0x3f80;                      // 1.0 in bfloat16
  const s4 x = {one, (short)(one - (t & 7)), one, one};
  f4 acc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = f4{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(x, x, acc[k], 0, 0, 0);
  }
  f4 s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  out[t] = (s[0] + s[1]) + (s[2] + s[3]);
}

__global__ __launch_bounds__(kCalibThreads) void calib_mfma_f32(int iters, float* __restrict__ out) {
  const int t = blockIdx.x * kCalibThreads + threadIdx.x;
  const float x = 1.f + 1e-3f * (float)(t & 7);
  f4 acc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = f4{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, x, acc[k], 0, 0, 0);
  }
  f4 s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  out[t] = (s[0] + s[1]) + (s[2] + s[3]);
}

}  // namespace

int calib_elements() { return kCalibBlocks * kCalibThreads; }

hipError_t launch_calibrate(int kind, int iters, float* out, double* flops, hipStream_t s) {
  const double waves = (double)kCalibBlocks * kCalibThreads / 64;
  switch (kind) {
    case 0:
      hipLaunchKernelGGL(calib_fma, dim3(kCalibBlocks), dim3(kCalibThreads), 0, s, iters, out);
      *flops = (double)kCalibBlocks * kCalibThreads * iters * 4 * 8 * 2;
      break;
    case 1:
      hipLaunchKernelGGL(calib_mfma_bf16, dim3(kCalibBlocks), dim3(kCalibThreads), 0, s, iters, out);
      *flops = waves * iters * 16 * (2.0 * 16 * 16 * 16);
      break;
    case 2:
      hipLaunchKernelGGL(calib_mfma_f32, dim3(kCalibBlocks), dim3(kCalibThreads), 0, s, iters, out);
      *flops = waves * iters * 16 * (2.0 * 16 * 16 * 4);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace taser
