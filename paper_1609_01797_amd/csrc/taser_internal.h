// Internal declarations shared by the HIP translation units of libtaser.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/taser.h"

namespace taser {

constexpr int kWave = 64;

// Flat argument block for the staged kernels (plain pointers and sizes).
struct StagedArgs {
  int32_t V, B, U, N, mod, mode, y_per_H, t_max, flags, tau_mode;
  float alpha;
  const float2* H;     // coherent channel matrices
  const float2* y;     // coherent receive vectors, or JED blocks Y
  const float2* s0;    // JED pilots
  float* Tt;           // [V][N][N]
  float* D;            // [V][N]
  float* lam;          // [V]
  float* tau;          // [V]
  int32_t* status;     // [V]
};

// Launchers (return hipSuccess or the launch error).
hipError_t launch_build_T(const StagedArgs& a, hipStream_t s);
// taser_build_T through the per-vector preprocessing (N - 1 <= 64, U <= 32):
// tiles > 0 when it applies.
int build_T_vec_tiles(const StagedArgs& a);
hipError_t launch_build_T_vec(const StagedArgs& a, hipStream_t s);
hipError_t launch_solve(const StagedArgs& a, const float* Tt, const float* D, const float* tau,
                        float* L, int32_t* status, hipStream_t s);
hipError_t launch_detect(int32_t V, int32_t N, const float* L, const float* D, int8_t* sbar,
                         float* margin, hipStream_t s);

// Fused single-launch detector for N-1 in {16, 32, 64}.
struct FusedArgs {
  int32_t V, B, U, N, mod, mode, y_per_H, t_max, flags, tau_mode, prec;
  float alpha;
  const float2* H;
  const float2* y;
  const float2* s0;
  const float* tau_in;
  int8_t* sbar;
  float* margin;
  int32_t* status;
  float* L_out;
  float* ws;           // workspace, fused_workspace_bytes(a) bytes
};
bool fused_supported(const FusedArgs& a);        // group or per-vector kernel applies
bool fused_group_supported(const FusedArgs& a);  // 16 vectors share one channel (two kernels)
int fused_vec_tiles(const FusedArgs& a);         // per-vector kernel tile count, 0 = no
hipError_t launch_fused_vec(const FusedArgs& a, hipStream_t s);
size_t fused_workspace_bytes(const FusedArgs& a);
// File-scope device state of taser_run_static (run_static.hip): its size and
// the current device's address of it.
size_t static_scratch_bytes();
hipError_t static_scratch(void** ptr);
hipError_t launch_fused(const FusedArgs& a, hipStream_t s);
hipError_t launch_fused_prep(const FusedArgs& a, hipStream_t s);
hipError_t launch_fused_solve(const FusedArgs& a, hipStream_t s);
// Bytes of preparation-to-solve state per channel group of 16 vectors.
constexpr size_t kGroupWsBytes = 4352;
hipError_t launch_fused_tau(const FusedArgs& a, float* tau, hipStream_t s);
int calib_elements();
hipError_t launch_jed_channel(int V, int B, int K, bool qpsk, const void* Y, const void* s0,
                              const int8_t* sbar, void* h, hipStream_t s);
hipError_t launch_calibrate(int kind, int iters, float* out, double* flops, hipStream_t s);

// Fixed-point Algorithm 1 (Section IV-C), N <= 64.  Inputs: words That
// [V][N][N] and D [V][N], or (Tt set) the float32 T~ [V][N][N], D [V][N] and
// tau [V] quantised in the kernel.  Outputs: words L and / or real values Lf
// [V][N(N+1)/2], decisions sbar [V][N-1] (or NULL), status [V] (in / out).
struct FixedArgs {
  int32_t V, N, t_max;
  const int16_t* That;
  const int16_t* D;
  const float* Tt;
  const float* Df;
  const float* tau;
  int16_t* L;
  float* Lf;
  int8_t* sbar;
  int32_t* status;
};
hipError_t launch_fixed_quantize(const FixedArgs& a, const float* Tt, const float* D,
                                 const float* tau, int16_t* That, int16_t* Dq, hipStream_t s);
hipError_t launch_fixed_solve(const FixedArgs& a, hipStream_t s);

// Reference detectors of the comparison (Section V-A): matched filter, MMSE,
// exhaustive ML, K-best.  M = N - 1 real dimensions.
struct RefArgs {
  int32_t V, B, U, M, mod, y_per_H, kind, K;
  float n0;
  const float2* H;
  const float2* y;
  int8_t* sbar;        // [V][M]
  float* soft;         // MF / MMSE: [V][M] estimates; ML / K-best: [V] residual; or NULL
};
hipError_t launch_reference(const RefArgs& a, hipStream_t s);

// Exact SDR of eq. (7) in float64, one workgroup per vector, 2 <= N <= 65.
struct SdrArgs {
  int32_t V, N;
  const float* Tt;          // [V][N][N]
  const float* D;           // [V][N], or NULL when Tt holds T itself
  const int32_t* status;    // [V] or NULL: nonzero entries are skipped
  int8_t* sbar;             // [V][N-1]
  double* objective;        // [V] or NULL
  double* gap;              // [V] or NULL
  double* X;                // [V][N][N] or NULL
  int32_t* iterations;      // [V] or NULL
};
hipError_t launch_sdr(const SdrArgs& a, hipStream_t s);

// Mixed-size batches: per-vector sizes and offsets, and the bucket lists in
// the workspace (count[kMixedBuckets] then kMixedBuckets lists of V indices).
constexpr int kMixedBuckets = 3;
struct MixedArgs {
  const int32_t* Bv;
  const int32_t* Uv;
  const int32_t* modv;
  const int64_t* H_off;   // complex elements
  const int64_t* y_off;
  int32_t stride;         // sbar / margin row stride
  int32_t* count;
  int32_t* list;
};
size_t mixed_workspace_bytes(int V);
hipError_t launch_mixed(const FusedArgs& a, const MixedArgs& m, const taser_mixed_launch_t* launch,
                        hipStream_t s);

// Unfolded variant (per-iteration step sizes) and its adjoint.
struct UnfoldedArgs {
  int32_t V, N, t_max, real, ckpt_every, flags;
};
size_t unfolded_lds_bytes(const UnfoldedArgs& a);
size_t unfolded_workspace_bytes(const UnfoldedArgs& a);
hipError_t launch_unfolded_forward(const UnfoldedArgs& a, const void* Tt, const void* D,
                                   const void* lam, const void* alpha, void* ckpt, void* Lout,
                                   hipStream_t s);
hipError_t launch_unfolded_backward(const UnfoldedArgs& a, const void* Tt, const void* D,
                                    const void* lam, const void* alpha, const void* ckpt,
                                    const void* dL, void* dalpha, void* ws, hipStream_t s);
// LDS bytes of `states` states of an N x N lower-triangular matrix stored as
// packed rows, row i padded to 4 * floor((i + 4) / 4) entries.
inline size_t unfolded_lds_states(int N, int states, size_t elem) {
  size_t s = 0;
  for (int r = 0; r < N; ++r) s += 4 * (size_t)((r + 4) / 4);
  return (size_t)states * s * elem;
}
// Vectors per wave of the unfolded kernels: two when every column that
// changes fits in 32 lanes (N <= 32, or N = 33 with L~_NN held), float only.
inline int unfolded_vectors_per_wave(const UnfoldedArgs& a) {
  const bool pin = !(a.flags & TASER_FLAG_LITERAL_LAST);
  return a.real == 0 && (a.N <= 32 || (a.N == 33 && pin)) ? 2 : 1;
}
// Per register bucket NP (multiple of 8, >= N) and vectors per wave HV;
// instantiated for float (HV = 1, 2) and double (HV = 1).
template <int NP, int HV, typename Real>
hipError_t unf_fwd(const UnfoldedArgs& a, const void* Tt, const void* D, const void* lam,
                   const void* alpha, void* ckpt, void* Lout, hipStream_t s);
template <int NP, int HV, typename Real>
hipError_t unf_bwd(const UnfoldedArgs& a, const void* Tt, const void* D, const void* lam,
                   const void* alpha, const void* ckpt, const void* dL, void* ws, hipStream_t s);

// LDS bytes the staged build kernel needs (0 if the shape does not fit).
size_t build_T_lds_bytes(int B, int U, int N);
size_t solve_lds_bytes(int N);

}  // namespace taser
