// Staged TASER kernels: preprocessing (T, D, T~, ||T~||_2, tau), Algorithm 1
// and slicing as three launches with T~ and L~ materialised in HBM.  They
// handle every problem size up to TASER_MAX_N and every mode; the fused
// kernel (fused.hip) is the fast path for the power-of-two shapes.
#include <math.h>

#include "spectral.h"
#include "taser_internal.h"

namespace taser {
namespace {

using spectral::hsqrt;
using spectral::kLanczosMax;
using spectral::rcp;
using spectral::rsq;
using spectral::wave_sum;

constexpr int kBuildThreads = 256;
constexpr int kLdsHBudget = 98304;   // bytes of LDS for the staged channel copy
constexpr int kLdsMax = 163840;      // LDS per workgroup on gfx950
// build_T_kernel's static LDS (two flags, the Lanczos tridiagonal and the
// reorthogonalisation scratch) is taken from the budget of its dynamic LDS
constexpr int kBuildStaticLds = 1280;
static_assert(2 * sizeof(int) + 2 * spectral::kLanczosMax * sizeof(float) +
                      spectral::lanczos_scratch_floats(TASER_MAX_N) * sizeof(float) <=
                  (size_t)kBuildStaticLds,
              "static LDS of build_T_kernel exceeds its reserve");

// One workgroup per vector.
//   phase 1: complex Gram G = H^H H, b = H^H y, ||y||^2 (JED: H := Y_r,
//            y := y_0 s_0) accumulated from an LDS copy of the channel;
//   phase 2: T (eq. (2) / eq. (5)) from G and b, D, T~ (Section III-C);
//   phase 3: ||T~||_2 by Lanczos with full reorthogonalisation and a
//            multisection of the Ritz tridiagonal, tau = alpha/||T~||_2.
__global__ __launch_bounds__(kBuildThreads) void build_T_kernel(StagedArgs a) {
  extern __shared__ float smem[];
  const int v = blockIdx.x;
  const int tid = threadIdx.x;
  const int B = a.B, U = a.U, N = a.N;
  const bool jed = a.mode == TASER_JED;
  const bool qpsk = a.mod == TASER_QPSK;

  // LDS: [channel copy | Lanczos basis] (shared region), then T and D.
  // channel columns padded to B + 1 entries: the threads of a wave read
  // different columns at the same row, which would otherwise share a bank
  const int BP = B + 1;
  const size_t hbytes = (size_t)BP * (U + 1) * sizeof(float2);
  const size_t qbytes = (size_t)spectral::lanczos_steps(N, false) * N * sizeof(float);
  const size_t region0 = hbytes > qbytes ? hbytes : qbytes;
  float2* Hc = reinterpret_cast<float2*>(smem);        // [U][BP] column-major channel
  float2* yc = Hc + (size_t)U * BP;                     // [B]
  float* T = reinterpret_cast<float*>(reinterpret_cast<char*>(smem) + region0);  // [N][N]
  float* Dl = T + (size_t)N * N;                        // [N]
  __shared__ int flag_nonfinite, flag_degenerate;

  if (tid == 0) { flag_nonfinite = 0; flag_degenerate = 0; }
  if (!jed) {
    const float2* Hg = a.H + (size_t)(v / a.y_per_H) * B * U;
    for (int e = tid; e < B * U; e += kBuildThreads) {
      const int b = e / U, u = e - b * U;
      Hc[(size_t)u * BP + b] = Hg[e];
    }
    const float2* yg = a.y + (size_t)v * B;
    for (int b = tid; b < B; b += kBuildThreads) yc[b] = yg[b];
  } else {
    const float2* Yg = a.y + (size_t)v * (U + 1) * B;
    const float2 s0 = a.s0[v];
    for (int e = tid; e < U * B; e += kBuildThreads) {   // slots 1..K
      const int u = e / B, b = e - u * B;
      Hc[(size_t)u * BP + b] = Yg[B + e];
    }
    for (int b = tid; b < B; b += kBuildThreads) {
      const float2 y0 = Yg[b];
      yc[b] = make_float2(y0.x * s0.x - y0.y * s0.y, y0.x * s0.y + y0.y * s0.x);
    }
  }
  __syncthreads();

  const float sg = jed ? -1.f : 1.f;
  const int n_pairs = U * (U + 1) / 2;
  const int n_entries = n_pairs + U + 1;
  for (int e = tid; e < n_entries; e += kBuildThreads) {
    float re = 0.f, im = 0.f;
    if (e < n_pairs) {
      // e -> (p, q), p >= q
      int p = (int)((sqrtf(8.f * (float)e + 1.f) - 1.f) * 0.5f);
      while (p * (p + 1) / 2 > e) --p;
      while ((p + 1) * (p + 2) / 2 <= e) ++p;
      const int q = e - p * (p + 1) / 2;
      const float2* hp = Hc + (size_t)p * BP;
      const float2* hq = Hc + (size_t)q * BP;
      for (int b = 0; b < B; ++b) {          // conj(h_p) h_q
        re += hp[b].x * hq[b].x + hp[b].y * hq[b].y;
        im += hp[b].x * hq[b].y - hp[b].y * hq[b].x;
      }
      const float gre = sg * re, gim = sg * im;
      if (qpsk) {
        T[p * N + q] = gre; T[q * N + p] = gre;
        T[(U + p) * N + U + q] = gre; T[(U + q) * N + U + p] = gre;
        T[p * N + U + q] = -gim; T[(U + q) * N + p] = -gim;
        if (p != q) { T[q * N + U + p] = gim; T[(U + p) * N + q] = gim; }
      } else {
        T[p * N + q] = gre; T[q * N + p] = gre;
      }
    } else if (e < n_pairs + U) {
      const int p = e - n_pairs;
      const float2* hp = Hc + (size_t)p * BP;
      for (int b = 0; b < B; ++b) {          // conj(h_p) y
        re += hp[b].x * yc[b].x + hp[b].y * yc[b].y;
        im += hp[b].x * yc[b].y - hp[b].y * yc[b].x;
      }
      // last column: -Hbar^T ybar in both modes
      T[p * N + (N - 1)] = -re; T[(N - 1) * N + p] = -re;
      if (qpsk) { T[(U + p) * N + (N - 1)] = -im; T[(N - 1) * N + U + p] = -im; }
    } else {
      for (int b = 0; b < B; ++b) re += yc[b].x * yc[b].x + yc[b].y * yc[b].y;
      T[(N - 1) * N + (N - 1)] = sg * re;
    }
  }
  __syncthreads();

  for (int e = tid; e < N * N; e += kBuildThreads)
    if (!isfinite(T[e])) flag_nonfinite = 1;
  __syncthreads();
  const bool nonfinite = flag_nonfinite != 0;
  for (int k = tid; k < N; k += kBuildThreads) {
    const float d = nonfinite ? 0.f : fabsf(T[k * N + k]);
    if (d == 0.f) flag_degenerate = 1;
    Dl[k] = d == 0.f ? 1.f : hsqrt(d);
  }
  __syncthreads();
  float* Ttg = a.Tt + (size_t)v * N * N;
  for (int e = tid; e < N * N; e += kBuildThreads) {
    const int i = e / N, j = e - i * N;
    const float t = nonfinite ? 0.f : T[e] * rcp(Dl[i] * Dl[j]);
    T[e] = t;
    Ttg[e] = t;
  }
  for (int k = tid; k < N; k += kBuildThreads) a.D[(size_t)v * N + k] = Dl[k];
  __syncthreads();

  // ---- ||T~||_2 (first wave only) ----
  float* Q = reinterpret_cast<float*>(smem);            // reuses the channel copy: [m][N]
  __shared__ float al[kLanczosMax], be2[kLanczosMax];
  __shared__ float lz[spectral::lanczos_scratch_floats(TASER_MAX_N)];
  if (tid < kWave) {
    const int lane = tid;
    const float lam = spectral::lanczos_norm(T, N, qpsk, jed, Q, al, be2, lz);
    if (lane == 0) {
      a.lam[v] = lam;
      if (a.tau_mode == TASER_TAU_SPECTRAL) a.tau[v] = a.alpha / (lam > 0.f ? lam : 1.f);
      a.status[v] = nonfinite ? TASER_VEC_NONFINITE : (flag_degenerate ? TASER_VEC_DEGENERATE : 0);
    }
  }
}

__device__ inline int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Algorithm 1 for one vector per workgroup; thread j owns column j of L~.
// LDS: T~ lower triangle, L~ and V, all packed.
__global__ __launch_bounds__(192) void solve_kernel(int N, int t_max, int flags,
                                                    const float* __restrict__ Ttg,
                                                    const float* __restrict__ Dg,
                                                    const float* __restrict__ taug,
                                                    float* __restrict__ Lg,
                                                    int32_t* __restrict__ statusg) {
  extern __shared__ float smem[];
  const int P = N * (N + 1) / 2;
  float* Tp = smem;
  float* Lp = Tp + P;
  float* Vp = Lp + P;
  __shared__ int st_bits;
  const int v = blockIdx.x;
  const int j = threadIdx.x;
  const float* Ttv = Ttg + (size_t)v * N * N;
  const float* Dv = Dg + (size_t)v * N;
  const int st_in = statusg[v];
  const bool skip = (st_in & (TASER_VEC_DEGENERATE | TASER_VEC_NONFINITE)) != 0;
  const bool pin = !(flags & TASER_FLAG_LITERAL_LAST);
  if (j == 0) st_bits = 0;
  for (int e = j; e < N * N; e += blockDim.x) {
    const int r = e / N, c = e - r * N;
    if (c <= r) Tp[tri(r, c)] = Ttv[e];
  }
  for (int e = j; e < P; e += blockDim.x) Lp[e] = 0.f;
  __syncthreads();
  const float Dj = j < N ? Dv[j] : 0.f;
  if (j < N) Lp[tri(j, j)] = Dj;
  __syncthreads();
  const float two_tau = 2.f * taug[v];
  const int iters = skip ? 0 : t_max;
  int my_bits = 0;
  for (int t = 0; t < iters; ++t) {
    if (j < N) {
      for (int i = j; i < N; ++i) {
        float acc = 0.f;
        for (int k = 0; k <= i; ++k) {
          const float tkj = k >= j ? Tp[tri(k, j)] : Tp[tri(j, k)];
          acc += Lp[tri(i, k)] * tkj;
        }
        Vp[tri(i, j)] = Lp[tri(i, j)] - two_tau * acc;
      }
    }
    __syncthreads();
    if (j < N) {
      if (j == N - 1) {
        const float vnn = Vp[tri(j, j)];
        if (!(vnn > 0.f)) my_bits |= TASER_VEC_VNN_NONPOS;
        if (pin) {
          Lp[tri(j, j)] = Dj;
        } else if (vnn != 0.f && isfinite(vnn)) {
          Lp[tri(j, j)] = vnn * (Dj / fabsf(vnn));
        } else {
          Lp[tri(j, j)] = Dj;
          my_bits |= TASER_VEC_ZERO_NORM;
        }
      } else {
        float nsq = 0.f;
        for (int i = j; i < N; ++i) { const float x = Vp[tri(i, j)]; nsq += x * x; }
        if (nsq > 0.f && isfinite(nsq)) {
          const float s = Dj * rsq(nsq);
          for (int i = j; i < N; ++i) Lp[tri(i, j)] = Vp[tri(i, j)] * s;
        } else {
          Lp[tri(j, j)] = Dj;
          for (int i = j + 1; i < N; ++i) Lp[tri(i, j)] = 0.f;
          my_bits |= TASER_VEC_ZERO_NORM;
        }
      }
    }
    __syncthreads();
  }
  if (my_bits) atomicOr(&st_bits, my_bits);
  float* Lv = Lg + (size_t)v * P;
  for (int e = j; e < P; e += blockDim.x) Lv[e] = Lp[e];
  __syncthreads();
  if (j == 0 && st_bits) statusg[v] = st_in | st_bits;
}

__global__ void detect_kernel(int32_t V, int32_t N, const float* __restrict__ L,
                              const float* __restrict__ D, int8_t* __restrict__ sbar,
                              float* __restrict__ margin) {
  const int P = N * (N + 1) / 2;
  const long long total = (long long)V * (N - 1);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long v = e / (N - 1);
    const int k = (int)(e - v * (N - 1));
    const float x = L[v * P + tri(N - 1, k)];
    sbar[e] = x >= 0.f ? (int8_t)1 : (int8_t)-1;
    if (margin) margin[e] = x / D[v * N + k];
  }
}

}  // namespace

size_t build_T_lds_bytes(int B, int U, int N) {
  const size_t hbytes = (size_t)(B + 1) * (U + 1) * sizeof(float2);
  if (hbytes > (size_t)kLdsHBudget) return 0;
  // the basis of the longer (real, BPSK) step rule
  size_t q = (size_t)spectral::lanczos_steps(N, false) * N * sizeof(float);
  size_t first = hbytes > q ? hbytes : q;
  const size_t total = first + (size_t)N * N * sizeof(float) + (size_t)N * sizeof(float);
  return total <= (size_t)(kLdsMax - kBuildStaticLds) ? total : 0;
}

size_t solve_lds_bytes(int N) { return 3 * (size_t)(N * (N + 1) / 2) * sizeof(float); }

hipError_t launch_build_T(const StagedArgs& a, hipStream_t s) {
  const size_t lds = build_T_lds_bytes(a.B, a.U, a.N);
  hipError_t e = hipFuncSetAttribute((const void*)build_T_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(build_T_kernel, dim3(a.V), dim3(kBuildThreads), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_solve(const StagedArgs& a, const float* Tt, const float* D, const float* tau,
                        float* L, int32_t* status, hipStream_t s) {
  const size_t lds = solve_lds_bytes(a.N);
  hipError_t e = hipFuncSetAttribute((const void*)solve_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int threads = ((a.N + kWave - 1) / kWave) * kWave;
  hipLaunchKernelGGL(solve_kernel, dim3(a.V), dim3(threads), lds, s, a.N, a.t_max, a.flags, Tt,
                     D, tau, L, status);
  return hipGetLastError();
}

hipError_t launch_detect(int32_t V, int32_t N, const float* L, const float* D, int8_t* sbar,
                         float* margin, hipStream_t s) {
  const long long total = (long long)V * (N - 1);
  long long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(detect_kernel, dim3((unsigned)blocks), dim3(256), 0, s, V, N, L, D, sbar,
                     margin);
  return hipGetLastError();
}

}  // namespace taser
