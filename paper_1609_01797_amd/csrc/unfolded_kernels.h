// Kernels of the unfolded TASER path (included by the unfolded_*.hip
// translation units, one per register bucket group).
//
// Unfolded TASER: Algorithm 1 with one step size per iteration,
// tau_t = alpha_t / ||T~||_2, and its adjoint with respect to alpha.
//
// Forward, iteration t (Section III-B/C):  V = L - tril(2 tau_t L T~),
// L' = prox(V), column k of L' = D_kk V_:,k / ||V_:,k||, L'_NN = D_NN.
// Adjoint, given the gradient Lb' of L':
//   prox:     Vb_:,k = (D_kk / n_k) (Lb'_:,k - u_k (u_k^T Lb'_:,k)),  u_k = V_:,k / n_k
//             (the held entry L_NN passes no gradient)
//   gradient: Lb = Vb - 2 tau_t tril(Vb T~)          (the forward's own product)
//   step:     taub_t = -2 <Vb, tril(L T~)>,  alphab_t = taub_t / ||T~||_2
// L is stored every c iterations; the backward pass recomputes each segment
// of c states from its checkpoint.
//
// One wave per vector.  Lane j owns column j: it holds column j of T~ in
// registers and produces column j of every product, V_ij = L_ij -
// 2 tau sum_k L_ik T~_kj, reading row i of L (or of Vb) from LDS as a
// broadcast (every lane reads the same address) and writing V_ij back to
// LDS.  Column norms, the prox and its adjoint are then lane-local
// (lane j touches only column j of V in LDS).  Rows and the triangular bounds of
// the sums are unrolled at compile time for a register bucket NP >= N
// (multiple of 8), which is also the LDS row stride, so every LDS address
// is a lane base plus a compile-time offset.  Real is
// float for training and double for gradient checks.
#pragma once

#include <math.h>

#include <type_traits>

#include "taser_internal.h"

namespace taser {
namespace unf {

// Occupancy request: the kernels keep `Arrays` register arrays of NP values
// (the column of T~; in the backward also the column of the adjoint Lb)
// plus working registers; asking for as many waves per SIMD as that budget
// allows keeps the compiler from hoisting every LDS row load into registers.
#ifndef TASER_UNF_REG_SLACK
#define TASER_UNF_REG_SLACK 100
#endif
template <int NP, typename Real, int Arrays>
constexpr int unf_waves() {
  const int regs = (Arrays * NP + TASER_UNF_REG_SLACK) * (int)(sizeof(Real) / 4);
  const int w = 512 / ((regs + 7) / 8 * 8);
  return w < 1 ? 1 : (w > 8 ? 8 : w);
}

template <int Begin, int End, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (Begin < End) {
    f(std::integral_constant<int, Begin>{});
    sfor<Begin + 1, End>(f);
  }
}

__host__ __device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }

template <typename Real>
__device__ __forceinline__ void load4(const Real* p, Real (&r)[4]) {
  if constexpr (sizeof(Real) == 4) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 x = *reinterpret_cast<const f4*>(p);
    r[0] = x[0]; r[1] = x[1]; r[2] = x[2]; r[3] = x[3];
  } else {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 x = *reinterpret_cast<const d2*>(p);
    const d2 y = *reinterpret_cast<const d2*>(p + 2);
    r[0] = x[0]; r[1] = x[1]; r[2] = y[0]; r[3] = y[1];
  }
}

template <typename Real>
__device__ __forceinline__ Real inv_sqrt(Real x) {
  if constexpr (sizeof(Real) == 8) return 1.0 / sqrt(x);
  else return 1.f / sqrtf(x);
}

template <typename Real>
__device__ __forceinline__ Real wave_sum(Real x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// For every row i < N: acc_i = sum_{k <= i} S[i][k] Tc[k] (S row-major with
// stride NP in LDS, zero above the diagonal), passed to emit(i, acc_i).
template <int NP, typename Real, typename F>
__device__ __forceinline__ void tril_rows(const Real* S, const Real (&Tc)[NP], int N, F&& emit) {
  constexpr int NS = NP;
  sfor<0, NP>([&](auto I) {
    constexpr int i = I;
    if (i < N) {
      Real a[4] = {0, 0, 0, 0};
      const Real* row = S + i * NS;
      sfor<0, i / 4 + 1>([&](auto KB) {
        constexpr int k = 4 * KB;
        Real r[4];
        load4(row + k, r);
        a[0] += r[0] * Tc[k];
        a[1] += r[1] * Tc[k + 1];
        a[2] += r[2] * Tc[k + 2];
        a[3] += r[3] * Tc[k + 3];
      });
      emit(I, (a[0] + a[1]) + (a[2] + a[3]));
      // keep the scheduler from hoisting later rows' loads above this row:
      // unbounded hoisting costs more registers than the latency it hides
      __builtin_amdgcn_sched_barrier(0);
    }
  });
}

// Packed lower-triangular rows in global memory <-> column j of a
// row-major LDS state (lanes N <= j < NP hold the zero padding columns).
template <int NP, typename Real>
__device__ __forceinline__ void lds_to_packed(Real* dst, const Real* S, int N, int j) {
  constexpr int NS = NP;
  Real* dj = dst + j;             // entry (i, j) at dj[i (i + 1) / 2]: static offsets
  const Real* Sj = S + j;
  sfor<0, NP>([&](auto I) {
    constexpr int i = I;
    if (i < N && i >= j) dj[i * (i + 1) / 2] = Sj[i * NS];
  });
}

template <int NP, typename Real>
__device__ __forceinline__ void packed_to_lds(Real* S, const Real* src, int N, int j) {
  constexpr int NS = NP;
  const Real* sj = src + j;
  Real* Sj = S + j;
  if (j < NS) {
    sfor<0, NP>([&](auto I) {
      constexpr int i = I;
      if (i < N) Sj[i * NS] = (i >= j && j < N) ? sj[i * (i + 1) / 2] : (Real)0;
    });
  }
}

// Column j of the prox (Section III-C) applied in place to the LDS state W:
// scale to norm D_jj, or hold (L_NN) / reset (zero or non-finite norm) to
// D_jj e_j.
template <int NP, typename Real>
__device__ __forceinline__ void prox_col(Real* W, int N, int j, Real nsq, Real Dj, bool pin) {
  constexpr int NS = NP;
  if (j >= N) return;
  if (!(pin && j == N - 1) && nsq > 0 && isfinite(nsq)) {
    const Real sc = Dj * inv_sqrt(nsq);
    sfor<0, NP>([&](auto I) {
      constexpr int i = I;
      if (i < N && i >= j) W[i * NS + j] *= sc;
    });
  } else {
    sfor<0, NP>([&](auto I) {
      constexpr int i = I;
      if (i < N && i >= j) W[i * NS + j] = i == j ? Dj : (Real)0;
    });
  }
}

// One forward iteration from the LDS state S (L_t) into W (L_{t+1}):
// W = prox(S - tril(2 tau S T~)).  Ends with a barrier.
template <int NP, typename Real>
__device__ __forceinline__ void fwd_step(const Real* S, Real* W, const Real (&Tc)[NP], int N,
                                         int j, Real tau2, Real Dj, bool pin) {
  constexpr int NS = NP;
  Real nsq = 0;
  tril_rows<NP>(S, Tc, N, [&](auto I, Real acc) {
    constexpr int i = I;
    const Real v = (i >= j && j < N) ? S[i * NS + j] - tau2 * acc : (Real)0;
    nsq += v * v;
    if (j < NS) W[i * NS + j] = v;
  });
  prox_col<NP>(W, N, j, nsq, Dj, pin);
  __syncthreads();
}

template <int NP, typename Real>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(unf_waves<NP, Real, 1>())))
void unf_forward(UnfoldedArgs a, const Real* __restrict__ Tt, const Real* __restrict__ D,
                 const Real* __restrict__ lam, const Real* __restrict__ alpha,
                 Real* __restrict__ ckpt, Real* __restrict__ Lout) {
  extern __shared__ __align__(16) unsigned char raw[];
  Real* S = reinterpret_cast<Real*>(raw);
  const long long v = blockIdx.x;
  const int N = a.N, P = N * (N + 1) / 2, c = a.ckpt_every;
  constexpr int NS = NP;
  const int nck = (a.t_max + c - 1) / c;
  const int j = threadIdx.x;
  Real* W = S + NS * NS;
  Real Tc[NP];
  sfor<0, NP>([&](auto I) {
    constexpr int k = I;
    Tc[k] = (k < N && j < N) ? Tt[(v * N + k) * N + j] : (Real)0;
  });
  const Real Dj = j < N ? D[v * N + j] : (Real)0;
  if (j < NS) {
    sfor<0, NP>([&](auto I) {
      constexpr int i = I;
      if (i < N) S[i * NS + j] = (i == j && j < N) ? Dj : (Real)0;
    });
  }
  __syncthreads();
  const Real lv = lam[v] > 0 ? lam[v] : (Real)1;
  const bool pin = !(a.flags & TASER_FLAG_LITERAL_LAST);
  for (int t = 0; t < a.t_max; ++t) {
    if (t % c == 0) lds_to_packed<NP>(ckpt + (v * nck + t / c) * (long long)P, S, N, j);
    fwd_step<NP>(S, W, Tc, N, j, (Real)2 * (alpha[t] / lv), Dj, pin);
    Real* x = S; S = W; W = x;
  }
  lds_to_packed<NP>(Lout + v * (long long)P, S, N, j);
}

template <int NP, typename Real>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(unf_waves<NP, Real, 2>())))
void unf_backward(UnfoldedArgs a, const Real* __restrict__ Tt, const Real* __restrict__ D,
                  const Real* __restrict__ lam, const Real* __restrict__ alpha,
                  const Real* __restrict__ ckpt, const Real* __restrict__ dL,
                  Real* __restrict__ part) {
  extern __shared__ __align__(16) unsigned char raw[];
  Real* lds = reinterpret_cast<Real*>(raw);
  const long long v = blockIdx.x;
  const int N = a.N, P = N * (N + 1) / 2, c = a.ckpt_every;
  constexpr int NS = NP;
  const int nck = (a.t_max + c - 1) / c;
  const int j = threadIdx.x;
  Real* seg = lds;                     // c states L_t0 .. L_t0+c-1, NS x NS each
  Real* W = lds + c * NS * NS;         // V, then Vb, of the current step
  Real Tc[NP], Lb[NP];
  sfor<0, NP>([&](auto I) {
    constexpr int k = I;
    Tc[k] = (k < N && j < N) ? Tt[(v * N + k) * N + j] : (Real)0;
  });
  const Real Dj = j < N ? D[v * N + j] : (Real)0;
  const Real lv = lam[v] > 0 ? lam[v] : (Real)1;
  const bool pin = !(a.flags & TASER_FLAG_LITERAL_LAST);
  sfor<0, NP>([&](auto I) {
    constexpr int i = I;
    Lb[i] = (i < N && i >= j && j < N) ? dL[v * P + tri(i, j)] : (Real)0;
  });
  for (int sg = nck - 1; sg >= 0; --sg) {
    const int t0 = sg * c, t1 = min(t0 + c, a.t_max);
    __syncthreads();
    packed_to_lds<NP>(seg, ckpt + (v * nck + sg) * (long long)P, N, j);
    __syncthreads();
    for (int t = t0; t < t1 - 1; ++t) {
      Real* cur = seg + (t - t0) * NS * NS;
      fwd_step<NP>(cur, cur + NS * NS, Tc, N, j, (Real)2 * (alpha[t] / lv), Dj, pin);
    }
    for (int t = t1 - 1; t >= t0; --t) {
      const Real tau2 = (Real)2 * (alpha[t] / lv);
      const Real* Ls = seg + (t - t0) * NS * NS;
      // V of step t into W, with the sums the prox adjoint needs:
      // P = tril(L_t T~), <V, P>, <Lb, P>, ||V||^2, <V, Lb>
      Real VP = 0, LbP = 0, nsq = 0, VLb = 0;
      tril_rows<NP>(Ls, Tc, N, [&](auto I, Real acc) {
        constexpr int i = I;
        const Real vv = (i >= j && j < N) ? Ls[i * NS + j] - tau2 * acc : (Real)0;
        VP += vv * acc;
        LbP += Lb[i] * acc;
        nsq += vv * vv;
        VLb += vv * Lb[i];
        if (j < NS) W[i * NS + j] = vv;
      });
      Real taub = 0;
      if (j < N && !(pin && j == N - 1) && nsq > 0 && isfinite(nsq)) {
        // Vb = (D/n)(Lb - u (u^T Lb)), u = V/n;  <Vb, P> from the sums
        const Real inv = inv_sqrt(nsq), g = Dj * inv, ub = VLb * inv;
        sfor<0, NP>([&](auto I) {
          constexpr int i = I;
          if (i < N && i >= j) W[i * NS + j] = g * (Lb[i] - W[i * NS + j] * inv * ub);
        });
        taub = g * (LbP - inv * ub * VP);
      } else if (j < NS) {
        sfor<0, NP>([&](auto I) {   // held or reset column: no gradient
          constexpr int i = I;
          if (i < N) W[i * NS + j] = 0;
        });
      }
      taub = wave_sum(taub);
      if (j == 0) part[v * a.t_max + t] = (Real)(-2) * taub / lv;
      __syncthreads();
      // Lb = Vb - 2 tau tril(Vb T~)
      tril_rows<NP>(W, Tc, N, [&](auto I, Real acc) {
        constexpr int i = I;
        Lb[i] = (i >= j && j < N) ? W[i * NS + j] - tau2 * acc : (Real)0;
      });
      __syncthreads();
    }
  }
}

template <typename Real>
size_t fwd_lds(int N) {
  return unfolded_lds_states(N, 2, sizeof(Real));
}

template <typename Real>
size_t bwd_lds(int N, int c) {
  return unfolded_lds_states(N, c + 1, sizeof(Real));
}

template <typename K>
hipError_t set_lds(K kernel, size_t lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int NP, typename Real>
hipError_t fwd_np(const UnfoldedArgs& a, const void* Tt, const void* D, const void* lam,
                  const void* alpha, void* ckpt, void* Lout, hipStream_t s) {
  const size_t lds = fwd_lds<Real>(a.N);
  hipError_t e = set_lds(unf_forward<NP, Real>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((unf_forward<NP, Real>), dim3(a.V), dim3(64), lds, s, a, (const Real*)Tt,
                     (const Real*)D, (const Real*)lam, (const Real*)alpha, (Real*)ckpt, (Real*)Lout);
  return hipGetLastError();
}

template <int NP, typename Real>
hipError_t bwd_np(const UnfoldedArgs& a, const void* Tt, const void* D, const void* lam,
                  const void* alpha, const void* ckpt, const void* dL, void* ws, hipStream_t s) {
  const size_t lds = bwd_lds<Real>(a.N, a.ckpt_every);
  hipError_t e = set_lds(unf_backward<NP, Real>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((unf_backward<NP, Real>), dim3(a.V), dim3(64), lds, s, a, (const Real*)Tt,
                     (const Real*)D, (const Real*)lam, (const Real*)alpha, (const Real*)ckpt,
                     (const Real*)dL, (Real*)ws);
  return hipGetLastError();
}

}  // namespace unf

// Defined here; explicitly instantiated, one register bucket group per
// translation unit, in unfolded_f32_*.hip and unfolded_f64_*.hip.
template <int NP, typename Real>
hipError_t unf_fwd(const UnfoldedArgs& a, const void* Tt, const void* D, const void* lam,
                   const void* alpha, void* ckpt, void* Lout, hipStream_t s) {
  return unf::fwd_np<NP, Real>(a, Tt, D, lam, alpha, ckpt, Lout, s);
}

template <int NP, typename Real>
hipError_t unf_bwd(const UnfoldedArgs& a, const void* Tt, const void* D, const void* lam,
                   const void* alpha, const void* ckpt, const void* dL, void* ws, hipStream_t s) {
  return unf::bwd_np<NP, Real>(a, Tt, D, lam, alpha, ckpt, dL, ws, s);
}

}  // namespace taser
