// Unfolded TASER: host launchers (bucket dispatch, LDS sizes) and the
// fixed-order reduction of the per-vector step-size gradients.  The
// iteration kernels and their adjoint live in unfolded_kernels.h.
#include "taser_internal.h"

namespace taser {
namespace {

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

// Register bucket: N rounded up to a multiple of 8.
template <typename F>
hipError_t dispatch(int N, F&& f) {
  switch ((N + 7) / 8) {
    case 1: return f(std::integral_constant<int, 8>{});
    case 2: return f(std::integral_constant<int, 16>{});
    case 3: return f(std::integral_constant<int, 24>{});
    case 4: return f(std::integral_constant<int, 32>{});
    case 5: return f(std::integral_constant<int, 40>{});
    case 6: return f(std::integral_constant<int, 48>{});
    case 7: return f(std::integral_constant<int, 56>{});
    case 8: return f(std::integral_constant<int, 64>{});
    default: return hipErrorInvalidValue;
  }
}

template <typename Real>
hipError_t fwd(const UnfoldedArgs& a, const void* Tt, const void* D, const void* lam,
               const void* alpha, void* ckpt, void* Lout, hipStream_t s) {
  return dispatch(a.N, [&](auto np) {
    constexpr int NP = decltype(np)::value;
    if constexpr (sizeof(Real) == 4 && NP <= 40) {
      if (unfolded_vectors_per_wave(a) == 2)
        return unf_fwd<NP, 2, Real>(a, Tt, D, lam, alpha, ckpt, Lout, s);
    }
    return unf_fwd<NP, 1, Real>(a, Tt, D, lam, alpha, ckpt, Lout, s);
  });
}

template <typename Real>
hipError_t bwd(const UnfoldedArgs& a, const void* Tt, const void* D, const void* lam,
               const void* alpha, const void* ckpt, const void* dL, void* dalpha, void* ws,
               hipStream_t s) {
  // an empty batch launches only the reduction, which writes dalpha = 0
  hipError_t e = a.V == 0 ? hipSuccess : dispatch(a.N, [&](auto np) {
    constexpr int NP = decltype(np)::value;
    if constexpr (sizeof(Real) == 4 && NP <= 40) {
      if (unfolded_vectors_per_wave(a) == 2)
        return unf_bwd<NP, 2, Real>(a, Tt, D, lam, alpha, ckpt, dL, ws, s);
    }
    return unf_bwd<NP, 1, Real>(a, Tt, D, lam, alpha, ckpt, dL, ws, s);
  });
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(unf_reduce<Real>, dim3(a.t_max), dim3(256), 0, s, a.V, a.t_max,
                     (const Real*)ws, (Real*)dalpha);
  return hipGetLastError();
}

}  // namespace

size_t unfolded_lds_bytes(const UnfoldedArgs& a) {
  return unfolded_lds_states(a.N, (a.ckpt_every + 1) * unfolded_vectors_per_wave(a),
                             a.real == 1 ? 8 : 4);
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
