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
// Lane j of a vector owns column j: it holds column j of T~ in registers and
// produces column j of every product, V_ij = L_ij - 2 tau sum_k L_ik T~_kj,
// reading row i of L (or of Vb) from LDS as a broadcast and writing V_ij
// back to LDS, where the prox rescales its own column in place.  Column
// norms, the prox and its adjoint are then lane-local.  LDS states are
// packed lower-triangular rows, row i padded to a multiple of 4 entries, so
// the row offsets are compile-time constants.  Rows and the triangular
// bounds of the sums are unrolled at compile time for a register bucket
// NP >= N (multiple of 8).  HV vectors share a wave (64 / HV lanes each):
// two when every column but a held last one fits in 32 lanes.  Real is float
// for training and double for gradient checks.
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
constexpr int kRegSlack = 100;
template <int NP, typename Real, int Arrays>
constexpr int unf_waves() {
  const int regs = (Arrays * NP + kRegSlack) * (int)(sizeof(Real) / 4);
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

// Packed LDS rows: row i holds columns 0 .. rlen(i) - 1 (entries beyond the
// diagonal are zero) and starts at roff(i).
__host__ __device__ constexpr int rlen(int i) { return 4 * ((i + 4) / 4); }
__host__ __device__ constexpr int roff(int i) {
  int s = 0;
  for (int r = 0; r < i; ++r) s += rlen(r);
  return s;
}

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
  else return __builtin_amdgcn_rsqf(x);   // hardware rsqrt, about one ulp
}

// Sum over the CW lanes of one vector.
template <int CW, typename Real>
__device__ __forceinline__ Real vec_sum(Real x) {
  for (int off = CW / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// For every row i < N: acc_i = sum_{k <= i} S[i][k] Tc[k], passed to
// emit(i, acc_i).
template <int NP, typename Real, typename F>
__device__ __forceinline__ void tril_rows(const Real* S, const Real (&Tc)[NP], int N, F&& emit) {
  sfor<0, NP>([&](auto I) {
    constexpr int i = I;
    if (i < N) {
      Real a[4] = {0, 0, 0, 0};
      const Real* row = S + roff(i);
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

// Packed lower-triangular rows in global memory <-> column j of an LDS
// state (only the lanes that own a column, j < jc).
template <int NP, typename Real>
__device__ __forceinline__ void lds_to_packed(Real* dst, const Real* S, int N, int j, int jc) {
  if (j >= jc) return;
  Real* dj = dst + j;             // entry (i, j) at dj[i (i + 1) / 2]: static offsets
  const Real* Sj = S + j;
  sfor<0, NP>([&](auto I) {
    constexpr int i = I;
    if (i < N && i >= j) dj[i * (i + 1) / 2] = Sj[roff(i)];
  });
}

template <int NP, typename Real>
__device__ __forceinline__ void packed_to_lds(Real* S, const Real* src, int N, int j, int jc) {
  if (j >= jc) return;
  const Real* sj = src + j;
  Real* Sj = S + j;
  sfor<0, NP>([&](auto I) {
    constexpr int i = I;
    if (i < N && i >= j) Sj[roff(i)] = sj[i * (i + 1) / 2];
  });
}

// Column j of the prox (Section III-C) applied in place to the LDS state W:
// scale to norm D_jj, or hold (L_NN) / reset (zero or non-finite norm) to
// D_jj e_j.
template <int NP, typename Real>
__device__ __forceinline__ void prox_col(Real* W, int N, int j, int jc, Real nsq, Real Dj,
                                         bool pin) {
  if (j >= jc) return;
  Real* Wj = W + j;
  if (!(pin && j == N - 1) && nsq > 0 && isfinite(nsq)) {
    const Real sc = Dj * inv_sqrt(nsq);
    sfor<0, NP>([&](auto I) {
      constexpr int i = I;
      if (i < N && i >= j) Wj[roff(i)] *= sc;
    });
  } else {
    sfor<0, NP>([&](auto I) {
      constexpr int i = I;
      if (i < N && i >= j) Wj[roff(i)] = i == j ? Dj : (Real)0;
    });
  }
}

// One forward iteration from the LDS state S (L_t) into W (L_{t+1}):
// W = prox(S - tril(2 tau S T~)).  Ends with a barrier.
template <int NP, typename Real>
__device__ __forceinline__ void fwd_step(const Real* S, Real* W, const Real (&Tc)[NP], int N,
                                         int j, int jc, Real tau2, Real Dj, bool pin) {
  Real nsq = 0;
  tril_rows<NP>(S, Tc, N, [&](auto I, Real acc) {
    constexpr int i = I;
    const Real v = (i >= j && j < jc) ? S[roff(i) + j] - tau2 * acc : (Real)0;
    nsq += v * v;
    if (j < jc && i >= j) W[roff(i) + j] = v;
  });
  prox_col<NP>(W, N, j, jc, nsq, Dj, pin);
  __syncthreads();
}

// Zero `states` LDS states of one vector (the padding above the diagonal
// stays zero from here on) and, when the lanes do not own the last column
// (it is held at D_NN), write that column once into every state.
template <typename Real>
__device__ __forceinline__ void init_states(Real* S, int states, int SS, int N, int CW, int j,
                                            bool held_last, Real DN) {
  for (int e = j; e < states * SS; e += CW) S[e] = 0;
  __syncthreads();
  if (held_last && j == 0)
    for (int s = 0; s < states; ++s) S[s * SS + roff(N - 1) + (N - 1)] = DN;
  __syncthreads();
}

template <int NP, int HV, typename Real>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(unf_waves<NP, Real, 1>())))
void unf_forward(UnfoldedArgs a, const Real* __restrict__ Tt, const Real* __restrict__ D,
                 const Real* __restrict__ lam, const Real* __restrict__ alpha,
                 Real* __restrict__ ckpt, Real* __restrict__ Lout) {
  constexpr int CW = 64 / HV;
  extern __shared__ __align__(16) unsigned char raw[];
  const int hv = threadIdx.x / CW, j = threadIdx.x % CW;
  const long long v = (long long)blockIdx.x * HV + hv;
  const bool live = v < a.V;
  const long long vv = live ? v : a.V - 1;       // an idle half mirrors a valid vector
  const int N = a.N, P = N * (N + 1) / 2, c = a.ckpt_every, SS = roff(N);
  const int nck = (a.t_max + c - 1) / c;
  const int jc = N < CW ? N : CW;                // lanes that own a column
  const bool pin = !(a.flags & TASER_FLAG_LITERAL_LAST);
  Real* S = reinterpret_cast<Real*>(raw) + hv * 2 * SS;
  Real* W = S + SS;
  Real Tc[NP];
  sfor<0, NP>([&](auto I) {
    constexpr int k = I;
    Tc[k] = (k < N && j < jc) ? Tt[(vv * N + k) * N + j] : (Real)0;
  });
  const Real Dj = j < jc ? D[vv * N + j] : (Real)0;
  const Real DN = D[vv * N + N - 1];
  init_states(S, 2, SS, N, CW, j, jc < N, DN);
  if (j < jc) S[roff(j) + j] = Dj;
  __syncthreads();
  const Real lv = lam[vv] > 0 ? lam[vv] : (Real)1;
  for (int t = 0; t < a.t_max; ++t) {
    if (t % c == 0 && live) {
      Real* dst = ckpt + (v * nck + t / c) * (long long)P;
      lds_to_packed<NP>(dst, S, N, j, jc);
      if (jc < N && j == 0) dst[P - 1] = DN;
    }
    fwd_step<NP>(S, W, Tc, N, j, jc, (Real)2 * (alpha[t] / lv), Dj, pin);
    Real* x = S; S = W; W = x;
  }
  if (live) {
    lds_to_packed<NP>(Lout + v * (long long)P, S, N, j, jc);
    if (jc < N && j == 0) Lout[v * (long long)P + P - 1] = DN;
  }
}

template <int NP, int HV, typename Real>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(unf_waves<NP, Real, 2>())))
void unf_backward(UnfoldedArgs a, const Real* __restrict__ Tt, const Real* __restrict__ D,
                  const Real* __restrict__ lam, const Real* __restrict__ alpha,
                  const Real* __restrict__ ckpt, const Real* __restrict__ dL,
                  Real* __restrict__ part) {
  constexpr int CW = 64 / HV;
  extern __shared__ __align__(16) unsigned char raw[];
  const int hv = threadIdx.x / CW, j = threadIdx.x % CW;
  const long long v = (long long)blockIdx.x * HV + hv;
  const bool live = v < a.V;
  const long long vv = live ? v : a.V - 1;
  const int N = a.N, P = N * (N + 1) / 2, c = a.ckpt_every, SS = roff(N);
  const int nck = (a.t_max + c - 1) / c;
  const int jc = N < CW ? N : CW;
  const bool pin = !(a.flags & TASER_FLAG_LITERAL_LAST);
  Real* seg = reinterpret_cast<Real*>(raw) + hv * (c + 1) * SS;   // c states, then Vb
  Real* W = seg + c * SS;
  Real Tc[NP], Lb[NP];
  sfor<0, NP>([&](auto I) {
    constexpr int k = I;
    Tc[k] = (k < N && j < jc) ? Tt[(vv * N + k) * N + j] : (Real)0;
  });
  const Real Dj = j < jc ? D[vv * N + j] : (Real)0;
  const Real DN = D[vv * N + N - 1];
  const Real lv = lam[vv] > 0 ? lam[vv] : (Real)1;
  sfor<0, NP>([&](auto I) {
    constexpr int i = I;
    Lb[i] = (i < N && i >= j && j < jc) ? dL[vv * P + tri(i, j)] : (Real)0;
  });
  // seg states hold the held last column; the Vb buffer keeps it at zero
  init_states(seg, c, SS, N, CW, j, jc < N, DN);
  for (int e = j; e < SS; e += CW) W[e] = 0;
  __syncthreads();
  for (int sg = nck - 1; sg >= 0; --sg) {
    const int t0 = sg * c, t1 = min(t0 + c, a.t_max);
    __syncthreads();
    packed_to_lds<NP>(seg, ckpt + (vv * nck + sg) * (long long)P, N, j, jc);
    __syncthreads();
    for (int t = t0; t < t1 - 1; ++t) {
      Real* cur = seg + (t - t0) * SS;
      fwd_step<NP>(cur, cur + SS, Tc, N, j, jc, (Real)2 * (alpha[t] / lv), Dj, pin);
    }
    for (int t = t1 - 1; t >= t0; --t) {
      const Real tau2 = (Real)2 * (alpha[t] / lv);
      const Real* Ls = seg + (t - t0) * SS;
      // V of step t into W, with the sums the prox adjoint needs:
      // P = tril(L_t T~), <V, P>, <Lb, P>, ||V||^2, <V, Lb>
      Real VP = 0, LbP = 0, nsq = 0, VLb = 0;
      tril_rows<NP>(Ls, Tc, N, [&](auto I, Real acc) {
        constexpr int i = I;
        const Real vv2 = (i >= j && j < jc) ? Ls[roff(i) + j] - tau2 * acc : (Real)0;
        VP += vv2 * acc;
        LbP += Lb[i] * acc;
        nsq += vv2 * vv2;
        VLb += vv2 * Lb[i];
        if (j < jc && i >= j) W[roff(i) + j] = vv2;
      });
      Real taub = 0;
      if (j < jc && !(pin && j == N - 1) && nsq > 0 && isfinite(nsq)) {
        // Vb = (D/n)(Lb - u (u^T Lb)), u = V/n;  <Vb, P> from the sums
        const Real inv = inv_sqrt(nsq), g = Dj * inv, ub = VLb * inv;
        Real* Wj = W + j;
        sfor<0, NP>([&](auto I) {
          constexpr int i = I;
          if (i < N && i >= j) Wj[roff(i)] = g * (Lb[i] - Wj[roff(i)] * inv * ub);
        });
        taub = g * (LbP - inv * ub * VP);
      } else if (j < jc) {
        Real* Wj = W + j;
        sfor<0, NP>([&](auto I) {   // held or reset column: no gradient
          constexpr int i = I;
          if (i < N && i >= j) Wj[roff(i)] = 0;
        });
      }
      taub = vec_sum<CW>(taub);
      if (j == 0 && live) part[v * a.t_max + t] = (Real)(-2) * taub / lv;
      __syncthreads();
      // Lb = Vb - 2 tau tril(Vb T~)
      tril_rows<NP>(W, Tc, N, [&](auto I, Real acc) {
        constexpr int i = I;
        Lb[i] = (i >= j && j < jc) ? W[roff(i) + j] - tau2 * acc : (Real)0;
      });
      __syncthreads();
    }
  }
}

template <typename Real>
size_t fwd_lds(int N, int hv) {
  return unfolded_lds_states(N, 2 * hv, sizeof(Real));
}

template <typename Real>
size_t bwd_lds(int N, int c, int hv) {
  return unfolded_lds_states(N, (c + 1) * hv, sizeof(Real));
}

template <typename K>
hipError_t set_lds(K kernel, size_t lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <int NP, int HV, typename Real>
hipError_t fwd_np(const UnfoldedArgs& a, const void* Tt, const void* D, const void* lam,
                  const void* alpha, void* ckpt, void* Lout, hipStream_t s) {
  const size_t lds = fwd_lds<Real>(a.N, HV);
  hipError_t e = set_lds(unf_forward<NP, HV, Real>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((unf_forward<NP, HV, Real>), dim3((a.V + HV - 1) / HV), dim3(64), lds, s, a,
                     (const Real*)Tt, (const Real*)D, (const Real*)lam, (const Real*)alpha,
                     (Real*)ckpt, (Real*)Lout);
  return hipGetLastError();
}

template <int NP, int HV, typename Real>
hipError_t bwd_np(const UnfoldedArgs& a, const void* Tt, const void* D, const void* lam,
                  const void* alpha, const void* ckpt, const void* dL, void* ws, hipStream_t s) {
  const size_t lds = bwd_lds<Real>(a.N, a.ckpt_every, HV);
  hipError_t e = set_lds(unf_backward<NP, HV, Real>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((unf_backward<NP, HV, Real>), dim3((a.V + HV - 1) / HV), dim3(64), lds, s,
                     a, (const Real*)Tt, (const Real*)D, (const Real*)lam, (const Real*)alpha,
                     (const Real*)ckpt, (const Real*)dL, (Real*)ws);
  return hipGetLastError();
}

}  // namespace unf

// Defined here; explicitly instantiated, one register bucket group per
// translation unit, in unfolded_f32_*.hip and unfolded_f64_*.hip.
template <int NP, int HV, typename Real>
hipError_t unf_fwd(const UnfoldedArgs& a, const void* Tt, const void* D, const void* lam,
                   const void* alpha, void* ckpt, void* Lout, hipStream_t s) {
  return unf::fwd_np<NP, HV, Real>(a, Tt, D, lam, alpha, ckpt, Lout, s);
}

template <int NP, int HV, typename Real>
hipError_t unf_bwd(const UnfoldedArgs& a, const void* Tt, const void* D, const void* lam,
                   const void* alpha, const void* ckpt, const void* dL, void* ws, hipStream_t s) {
  return unf::bwd_np<NP, HV, Real>(a, Tt, D, lam, alpha, ckpt, dL, ws, s);
}

}  // namespace taser
