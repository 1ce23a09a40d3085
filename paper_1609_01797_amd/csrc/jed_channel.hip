// Channel estimate of joint channel estimation and detection (Section II-B,
// eq. (4)): with the pilot s_0 and the detected data symbols s_1 .. s_K of a
// block, h = Y [s_0; s_r], i.e. h_b = sum_k Y[k][b] s_k over the K + 1 slots.
// One thread per (block, antenna): the B threads of a block read each slot's
// row of Y contiguously.
#include "taser_internal.h"

namespace taser {
namespace {

__global__ __launch_bounds__(256) void jed_channel_kernel(int V, int B, int K, int qpsk,
                                                          const float2* __restrict__ Y,
                                                          const float2* __restrict__ s0,
                                                          const int8_t* __restrict__ sbar,
                                                          float2* __restrict__ h) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long long)V * B) return;
  const long long v = t / B;
  const int b = (int)(t - v * B);
  const float2* Yv = Y + v * (long long)(K + 1) * B + b;
  const int8_t* sv = sbar + v * (long long)(qpsk ? 2 * K : K);
  const float2 p = s0[v];
  float2 y = Yv[0];
  float re = y.x * p.x - y.y * p.y, im = y.x * p.y + y.y * p.x;
  for (int k = 1; k <= K; ++k) {
    y = Yv[(long long)k * B];
    const float sr = (float)sv[k - 1];
    const float si = qpsk ? (float)sv[K + k - 1] : 0.f;
    re += y.x * sr - y.y * si;
    im += y.x * si + y.y * sr;
  }
  h[t] = make_float2(re, im);
}

}  // namespace

hipError_t launch_jed_channel(int V, int B, int K, bool qpsk, const void* Y, const void* s0,
                              const int8_t* sbar, void* h, hipStream_t s) {
  const long long n = (long long)V * B;
  hipLaunchKernelGGL(jed_channel_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, V, B,
                     K, qpsk ? 1 : 0, static_cast<const float2*>(Y),
                     static_cast<const float2*>(s0), sbar, static_cast<float2*>(h));
  return hipGetLastError();
}

}  // namespace taser
