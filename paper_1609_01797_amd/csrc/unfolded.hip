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
// of c states from its checkpoint.  One 64-lane workgroup per vector, lane j
// owning column j of L (N <= 64), everything else in LDS.  Real is float for
// training and double for the gradient check.
#include <math.h>

#include "taser_internal.h"

namespace taser {
namespace {

__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }

template <typename Real>
__device__ Real block_sum(Real x, Real* red) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

template <typename Real>
struct UnfLds {
  Real* T;     // [N][N]
  Real* seg;   // [c][P] states L_{t0} .. L_{t0+c-1}
  Real* V;     // [P]
  Real* Pm;    // [P]  tril(L T~)
  Real* Vb;    // [P]
  Real* Lb;    // [P]
};

template <typename Real>
__device__ __forceinline__ Real rsqrt_r(Real x) {
  if constexpr (sizeof(Real) == 8) return 1.0 / sqrt(x);
  else return 1.f / sqrtf(x);
}

// One forward iteration from Lin to Lout (may alias), keeping V and
// tril(L T~) in LDS.  Returns nothing; lane j owns column j.
template <typename Real>
__device__ void unf_step(const UnfLds<Real>& s, const Real* Lin, Real* Lout, int N, Real tau,
                         Real Dj, bool pin, bool keep_P) {
  const int j = threadIdx.x;
  if (j < N) {
    for (int i = j; i < N; ++i) {
      Real acc = 0;
      for (int k = 0; k <= i; ++k) acc += Lin[tri(i, k)] * s.T[k * N + j];
      s.V[tri(i, j)] = Lin[tri(i, j)] - (Real)2 * tau * acc;
      if (keep_P) s.Pm[tri(i, j)] = acc;
    }
  }
  __syncthreads();
  if (j < N) {
    if (pin && j == N - 1) {
      Lout[tri(j, j)] = Dj;
    } else {
      Real nsq = 0;
      for (int i = j; i < N; ++i) { const Real x = s.V[tri(i, j)]; nsq += x * x; }
      if (nsq > 0 && isfinite(nsq)) {
        const Real sc = Dj * rsqrt_r(nsq);
        for (int i = j; i < N; ++i) Lout[tri(i, j)] = s.V[tri(i, j)] * sc;
      } else {
        Lout[tri(j, j)] = Dj;
        for (int i = j + 1; i < N; ++i) Lout[tri(i, j)] = 0;
      }
    }
  }
  __syncthreads();
}

template <typename Real>
__device__ UnfLds<Real> carve(Real* lds, int N, int c) {
  const int P = N * (N + 1) / 2;
  UnfLds<Real> s;
  s.T = lds;
  s.seg = s.T + N * N;
  s.V = s.seg + c * P;
  s.Pm = s.V + P;
  s.Vb = s.Pm + P;
  s.Lb = s.Vb + P;
  return s;
}

template <typename Real>
__device__ void load_T(const UnfLds<Real>& s, const Real* Tt, long long v, int N) {
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) s.T[e] = Tt[v * N * N + e];
}

template <typename Real>
__global__ __launch_bounds__(64) void unf_forward(UnfoldedArgs a, const Real* __restrict__ Tt,
                                                  const Real* __restrict__ D,
                                                  const Real* __restrict__ lam,
                                                  const Real* __restrict__ alpha,
                                                  Real* __restrict__ ckpt, Real* __restrict__ Lout) {
  extern __shared__ __align__(16) unsigned char raw[];
  Real* lds = reinterpret_cast<Real*>(raw);
  const long long v = blockIdx.x;
  const int N = a.N, P = N * (N + 1) / 2, c = a.ckpt_every;
  const int nck = (a.t_max + c - 1) / c;
  UnfLds<Real> s = carve(lds, N, c);
  load_T(s, Tt, v, N);
  Real* L = s.seg;   // working state
  for (int e = threadIdx.x; e < P; e += blockDim.x) L[e] = 0;
  __syncthreads();
  const int j = threadIdx.x;
  const Real Dj = j < N ? D[v * N + j] : (Real)0;
  if (j < N) L[tri(j, j)] = Dj;
  __syncthreads();
  const Real lv = lam[v] > 0 ? lam[v] : (Real)1;
  const bool pin = !(a.flags & TASER_FLAG_LITERAL_LAST);
  for (int t = 0; t < a.t_max; ++t) {
    if (t % c == 0 && ckpt) {
      Real* dst = ckpt + (v * nck + t / c) * (long long)P;
      for (int e = threadIdx.x; e < P; e += blockDim.x) dst[e] = L[e];
    }
    unf_step(s, L, L, N, alpha[t] / lv, Dj, pin, false);
  }
  for (int e = threadIdx.x; e < P; e += blockDim.x) Lout[v * P + e] = L[e];
}

template <typename Real>
__global__ __launch_bounds__(64) void unf_backward(UnfoldedArgs a, const Real* __restrict__ Tt,
                                                   const Real* __restrict__ D,
                                                   const Real* __restrict__ lam,
                                                   const Real* __restrict__ alpha,
                                                   const Real* __restrict__ ckpt,
                                                   const Real* __restrict__ dL,
                                                   Real* __restrict__ part) {
  extern __shared__ __align__(16) unsigned char raw[];
  Real* lds = reinterpret_cast<Real*>(raw);
  const long long v = blockIdx.x;
  const int N = a.N, P = N * (N + 1) / 2, c = a.ckpt_every;
  const int nck = (a.t_max + c - 1) / c;
  UnfLds<Real> s = carve(lds, N, c);
  load_T(s, Tt, v, N);
  for (int e = threadIdx.x; e < P; e += blockDim.x) s.Lb[e] = dL[v * P + e];
  __syncthreads();
  const int j = threadIdx.x;
  const Real Dj = j < N ? D[v * N + j] : (Real)0;
  const Real lv = lam[v] > 0 ? lam[v] : (Real)1;
  const bool pin = !(a.flags & TASER_FLAG_LITERAL_LAST);
  for (int sg = nck - 1; sg >= 0; --sg) {
    const int t0 = sg * c, t1 = min(t0 + c, a.t_max);
    // recompute L_{t0} .. L_{t1-1} into seg[0 .. t1-t0-1]
    const Real* src = ckpt + (v * nck + sg) * (long long)P;
    for (int e = threadIdx.x; e < P; e += blockDim.x) s.seg[e] = src[e];
    __syncthreads();
    for (int t = t0; t < t1 - 1; ++t) {
      Real* cur = s.seg + (t - t0) * P;
      Real* nxt = cur + P;
      for (int e = threadIdx.x; e < P; e += blockDim.x) nxt[e] = 0;
      __syncthreads();
      unf_step(s, cur, nxt, N, alpha[t] / lv, Dj, pin, false);
    }
    // adjoint of iterations t1-1 .. t0 (iteration t maps L_t to L_{t+1})
    for (int t = t1 - 1; t >= t0; --t) {
      const Real tau = alpha[t] / lv;
      const Real* Lp = s.seg + (t - t0) * P;
      Real taub = 0;
      if (j < N) {
        for (int i = j; i < N; ++i) {
          Real acc = 0;
          for (int k = 0; k <= i; ++k) acc += Lp[tri(i, k)] * s.T[k * N + j];
          s.V[tri(i, j)] = Lp[tri(i, j)] - (Real)2 * tau * acc;
          s.Pm[tri(i, j)] = acc;
        }
        // prox backward for column j
        if (pin && j == N - 1) {
          s.Vb[tri(j, j)] = 0;
        } else {
          Real nsq = 0;
          for (int i = j; i < N; ++i) { const Real x = s.V[tri(i, j)]; nsq += x * x; }
          if (nsq > 0 && isfinite(nsq)) {
            const Real inv = rsqrt_r(nsq);
            Real ub = 0;
            for (int i = j; i < N; ++i) ub += s.V[tri(i, j)] * inv * s.Lb[tri(i, j)];
            const Real g = Dj * inv;
            for (int i = j; i < N; ++i) {
              const Real vb = g * (s.Lb[tri(i, j)] - s.V[tri(i, j)] * inv * ub);
              s.Vb[tri(i, j)] = vb;
              taub += vb * s.Pm[tri(i, j)];
            }
          } else {
            for (int i = j; i < N; ++i) s.Vb[tri(i, j)] = 0;   // reset column: no gradient
          }
        }
      }
      taub = block_sum(taub * (Real)(-2), (Real*)nullptr);
      if (threadIdx.x == 0) part[v * a.t_max + t] = taub / lv;
      __syncthreads();
      // Lb = Vb - 2 tau tril(Vb T~)
      if (j < N) {
        for (int i = j; i < N; ++i) {
          Real acc = 0;
          for (int k = 0; k <= i; ++k) acc += s.Vb[tri(i, k)] * s.T[k * N + j];
          s.Lb[tri(i, j)] = s.Vb[tri(i, j)] - (Real)2 * tau * acc;
        }
      }
      __syncthreads();
    }
  }
}

// dalpha[t] = sum over vectors of part[v][t], in a fixed order.
template <typename Real>
__global__ __launch_bounds__(256) void unf_reduce(int V, int t_max, const Real* __restrict__ part,
                                                  Real* __restrict__ out) {
  __shared__ Real red[256];
  const int t = blockIdx.x;
  Real acc = 0;
  for (int v = threadIdx.x; v < V; v += 256) acc += part[(long long)v * t_max + t];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[t] = red[0];
}

template <typename Real>
size_t lds_bytes(int N, int c) {
  const size_t P = (size_t)N * (N + 1) / 2;
  return ((size_t)N * N + (size_t)c * P + 4 * P) * sizeof(Real);
}

template <typename Real>
hipError_t fwd(const UnfoldedArgs& a, const void* Tt, const void* D, const void* lam,
               const void* alpha, void* ckpt, void* Lout, hipStream_t s) {
  const size_t lds = lds_bytes<Real>(a.N, a.ckpt_every);
  hipError_t e = hipFuncSetAttribute((const void*)unf_forward<Real>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(unf_forward<Real>, dim3(a.V), dim3(64), lds, s, a, (const Real*)Tt,
                     (const Real*)D, (const Real*)lam, (const Real*)alpha, (Real*)ckpt, (Real*)Lout);
  return hipGetLastError();
}

template <typename Real>
hipError_t bwd(const UnfoldedArgs& a, const void* Tt, const void* D, const void* lam,
               const void* alpha, const void* ckpt, const void* dL, void* dalpha, void* ws,
               hipStream_t s) {
  const size_t lds = lds_bytes<Real>(a.N, a.ckpt_every);
  hipError_t e = hipFuncSetAttribute((const void*)unf_backward<Real>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(unf_backward<Real>, dim3(a.V), dim3(64), lds, s, a, (const Real*)Tt,
                     (const Real*)D, (const Real*)lam, (const Real*)alpha, (const Real*)ckpt,
                     (const Real*)dL, (Real*)ws);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(unf_reduce<Real>, dim3(a.t_max), dim3(256), 0, s, a.V, a.t_max,
                     (const Real*)ws, (Real*)dalpha);
  return hipGetLastError();
}

}  // namespace

size_t unfolded_lds_bytes(const UnfoldedArgs& a) {
  return a.real == 1 ? lds_bytes<double>(a.N, a.ckpt_every) : lds_bytes<float>(a.N, a.ckpt_every);
}

size_t unfolded_workspace_bytes(const UnfoldedArgs& a) {
  return (size_t)a.V * a.t_max * (a.real == 1 ? 8 : 4);
}

hipError_t launch_unfolded_forward(const UnfoldedArgs& a, const void* Tt, const void* D,
                                   const void* lam, const void* alpha, void* ckpt, void* Lout,
                                   hipStream_t s) {
  return a.real == 1 ? fwd<double>(a, Tt, D, lam, alpha, ckpt, Lout, s)
                     : fwd<float>(a, Tt, D, lam, alpha, ckpt, Lout, s);
}

hipError_t launch_unfolded_backward(const UnfoldedArgs& a, const void* Tt, const void* D,
                                    const void* lam, const void* alpha, const void* ckpt,
                                    const void* dL, void* dalpha, void* ws, hipStream_t s) {
  return a.real == 1 ? bwd<double>(a, Tt, D, lam, alpha, ckpt, dL, dalpha, ws, s)
                     : bwd<float>(a, Tt, D, lam, alpha, ckpt, dL, dalpha, ws, s);
}

}  // namespace taser
