// Exact semidefinite relaxation (eq. (7)): min Tr(T S) subject to
// diag(S) = 1 and S positive semidefinite, then the signs of the leading
// eigenvector of S (Section II-C), for 2 <= N <= 65, in float64 (the
// vector units run it at the float32 rate, and the interior-point iterates
// need the resolution: near the optimum X is close to rank one).
//
// One workgroup per problem (one wave for N <= 64, two for N = 65); its
// matrices live in LDS (odd row stride, so that a lane-per-row access
// spreads over the banks) and thread i owns row or column i.  A primal-dual interior-point method with the HKM direction
// keeps X (diag(X) = 1) and y (Z = C - Diag(y) positive definite) feasible,
// with C = T / max|T_ij| (the argmin does not change).  Each iteration, with
// mu = <X, Z> / N and a target sigma mu on the central path (sigma = 0.5 at
// first, then (1 - a)^2 clipped to [0.1, 0.9] after a step of length a):
//   Z = L L^T (Cholesky), W = L^-1 (lane j solves for column j),
//   Zinv = W^T W, (X o Zinv) dy = 1 - sigma mu diag(Zinv) (Cholesky again),
//   dX = sigma mu Zinv - X + X Diag(dy) Zinv, symmetrised;
// each step length is the largest of 1, 0.8, 0.8^2, ... at which X + a dX
// (or C - Diag(y + a dy)) still factors, times 0.95.  The iteration stops
// when <X, Z> <= 1e-9 max(1, |<C, X>|), when a factorisation of Z or of the
// Schur matrix fails, when the gap is below 1e-6 max(1, |<C, X>|) and has not
// halved in eight steps (rounding floor of a degenerate problem), or after
// 100 steps.  The leading eigenvector of the final X comes from five
// trace-normalised squarings (X^32) and power iteration started from the
// last column of X.
#include <math.h>

#include "taser_internal.h"

namespace taser {
namespace {

using real = double;
constexpr real kSigma0 = 0.5;
constexpr real kSigmaMin = 0.1;
constexpr real kSigmaMax = 0.9;
constexpr int kStall = 8;
constexpr real kStallTol = 1e-6;
constexpr real kStepFraction = 0.95;
constexpr real kGapTol = 1e-9;
constexpr int kMaxIter = 100;
constexpr int kMaxTrials = 40;
constexpr int kSquarings = 5;
constexpr int kPowerIters = 64;

template <int NP>
struct SdrLds {
  static constexpr int LD = NP | 1;
  real C[NP * LD];   // scaled T
  real X[NP * LD];
  real A[NP * LD];   // Cholesky of Z, Zinv, dX (symmetrised), X powers
  real B[NP * LD];   // L^-1, Schur matrix, dX (unsymmetrised), step trials, X powers
  real v[NP];
  real red[2];       // per-wave partials of block reductions (two waves)
  int ok;
};

template <int NP>
constexpr int kThreads = NP <= 64 ? 64 : 128;

__device__ real wave_sum(real x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Sum (or maximum) over the workgroup, called by every thread at the same
// point; with two waves the partials meet in LDS between two barriers.
template <int NP>
__device__ real block_sum(real x, real* red) {
  x = wave_sum(x);
  if constexpr (kThreads<NP> == 64) {
    return x;
  } else {
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    return red[0] + red[1];
  }
}

template <int NP>
__device__ real block_max(real x, real* red) {
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  if constexpr (kThreads<NP> == 64) {
    return x;
  } else {
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    return fmax(red[0], red[1]);
  }
}

// In-place Cholesky of the leading N x N block (lower triangle); false when
// a pivot is not positive and finite.  Entries above the diagonal are left
// as they were.
// With two waves the column of L must be complete before the update reads
// it (one wave executes its LDS accesses in program order and needs no
// barrier there).
template <int LD, bool kTwoWaves>
__device__ bool chol(real* A, int N, int* ok) {
  const int i = threadIdx.x;
  __syncthreads();  // every thread has read the previous result
  if (i == 0) *ok = 1;
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    if (i == k) {
      const real d = A[k * LD + k];
      const bool good = d > 0.0 && isfinite(d);
      if (!good) *ok = 0;
      A[k * LD + k] = good ? sqrt(d) : 1.0;
    }
    __syncthreads();
    real lik = 0.0;
    if (i > k && i < N) {
      lik = A[i * LD + k] / A[k * LD + k];
      A[i * LD + k] = lik;
    }
    if constexpr (kTwoWaves) __syncthreads();
    if (i > k && i < N)
      for (int j = k + 1; j <= i; ++j) A[i * LD + j] -= lik * A[j * LD + k];
    __syncthreads();
  }
  return *ok != 0;
}

// dst = src * src / trace(src * src), row i in thread i.
template <int NP, int LD>
__device__ void square_normalised(const real* src, real* dst, int N, real* red) {
  const int i = threadIdx.x;
  real diag = 0.0;
  if (i < N)
    for (int j = 0; j < N; ++j) {
      real acc = 0.0;
      for (int k = 0; k < N; ++k) acc += src[i * LD + k] * src[k * LD + j];
      dst[i * LD + j] = acc;
      if (j == i) diag = acc;
    }
  const real tr = block_sum<NP>(diag, red);
  const real inv = tr > 0.0 && isfinite(tr) ? 1.0 / tr : 0.0;
  if (i < N)
    for (int j = 0; j < N; ++j) dst[i * LD + j] *= inv;
  __syncthreads();
}

template <int NP>
__global__ __launch_bounds__(kThreads<NP>) void sdr_kernel(SdrArgs a) {
  constexpr int LD = SdrLds<NP>::LD;
  __shared__ SdrLds<NP> s;
  const int i = threadIdx.x;
  const long long vec = blockIdx.x;
  const int N = a.N;
  const bool row = i < N;
  const bool skip = a.status && a.status[vec] != 0;
  const float* Tt = a.Tt + vec * (long long)N * N;
  const float* Dv = a.D ? a.D + vec * (long long)N : nullptr;

  // C = D T~ D (T itself when no D is given), scaled by 1 / max|C_ij|; X = I
  real mx = 0.0;
  if (row) {
    const real di = Dv ? (real)Dv[i] : 1.0;
    for (int j = 0; j < N; ++j) {
      const real tij = Tt[(long long)i * N + j];
      const real t = skip ? 0.0 : (Dv ? di * tij * (real)Dv[j] : tij);
      s.C[i * LD + j] = t;
      s.X[i * LD + j] = i == j ? 1.0 : 0.0;
      mx = fmax(mx, fabs(t));
    }
  }
  mx = block_max<NP>(mx, s.red);
  const bool run = !skip && mx > 0.0 && isfinite(mx);
  const real scale = run ? mx : 1.0;
  const real iscale = 1.0 / scale;
  real yi = 0.0;  // y_i in lane i
  if (row) {
    real off = 0.0;
    for (int j = 0; j < N; ++j) {
      s.C[i * LD + j] = run ? s.C[i * LD + j] * iscale : 0.0;
      if (j != i) off += fabs(s.C[i * LD + j]);
    }
    yi = s.C[i * LD + i] - off - 1.0;  // Z = C - Diag(y) strictly diagonally dominant
  }
  __syncthreads();

  int it = 0;
  real sigma = kSigma0;
  real hist[kStall];  // gaps of the last kStall iterations (ring)
#pragma unroll
  for (int q = 0; q < kStall; ++q) hist[q] = INFINITY;
  for (; run && it < kMaxIter; ++it) {
    real xz = 0.0, cx = 0.0;
    if (row)
      for (int j = 0; j < N; ++j) {
        const real z = s.C[i * LD + j] - (i == j ? yi : 0.0);
        s.A[i * LD + j] = z;
        xz += s.X[i * LD + j] * z;
        cx += s.X[i * LD + j] * s.C[i * LD + j];
      }
    xz = block_sum<NP>(xz, s.red);
    cx = block_sum<NP>(cx, s.red);
    const real ref = fmax(1.0, fabs(cx));
    if (xz <= kGapTol * ref) break;
    real old = hist[0];
#pragma unroll
    for (int q = 0; q < kStall - 1; ++q) hist[q] = hist[q + 1];
    hist[kStall - 1] = xz;
    if (xz <= kStallTol * ref && !(xz < 0.5 * old)) break;  // stalled at the rounding floor
    const real smu = sigma * xz / (real)N;
    __syncthreads();
    if (!chol<LD, (kThreads<NP> > 64)>(s.A, N, &s.ok)) break;
    // B = L^-1 (lower triangular): lane i forward-substitutes column i
    if (row)
      for (int r = 0; r < N; ++r) {
        real acc = r == i ? 1.0 : 0.0;
        for (int k = i; k < r; ++k) acc -= s.A[r * LD + k] * s.B[k * LD + i];
        s.B[r * LD + i] = r < i ? 0.0 : acc / s.A[r * LD + r];
      }
    __syncthreads();
    // A = Zinv = B^T B, column i in lane i
    if (row)
      for (int r = 0; r < N; ++r) {
        real acc = 0.0;
        for (int k = r > i ? r : i; k < N; ++k) acc += s.B[k * LD + r] * s.B[k * LD + i];
        s.A[r * LD + i] = acc;
      }
    __syncthreads();
    // Schur system (X o Zinv) dy = 1 - sigma mu diag(Zinv), solved in B / v
    if (row) {
      for (int j = 0; j < N; ++j) s.B[i * LD + j] = s.X[i * LD + j] * s.A[i * LD + j];
      s.v[i] = 1.0 - smu * s.A[i * LD + i];
    }
    __syncthreads();
    if (!chol<LD, (kThreads<NP> > 64)>(s.B, N, &s.ok)) break;
    for (int k = 0; k < N; ++k) {
      if (i == k) s.v[k] /= s.B[k * LD + k];
      __syncthreads();
      if (i > k && row) s.v[i] -= s.B[i * LD + k] * s.v[k];
      __syncthreads();
    }
    for (int k = N - 1; k >= 0; --k) {
      if (i == k) s.v[k] /= s.B[k * LD + k];
      __syncthreads();
      if (i < k) s.v[i] -= s.B[k * LD + i] * s.v[k];
      __syncthreads();
    }
    const real dyi = row ? s.v[i] : 0.0;
    // B = sigma mu Zinv - X + X Diag(dy) Zinv, column i in lane i
    if (row)
      for (int r = 0; r < N; ++r) {
        real acc = 0.0;
        for (int k = 0; k < N; ++k) acc += s.X[r * LD + k] * s.v[k] * s.A[k * LD + i];
        s.B[r * LD + i] = smu * s.A[r * LD + i] - s.X[r * LD + i] + acc;
      }
    __syncthreads();
    // A = dX = (B + B^T) / 2, zero diagonal (exact when dy solves its system)
    if (row)
      for (int j = 0; j < N; ++j)
        s.A[i * LD + j] = j == i ? 0.0 : 0.5 * (s.B[i * LD + j] + s.B[j * LD + i]);
    __syncthreads();
    // step lengths: backtrack until X + a dX, then C - Diag(y + a dy), factor
    real ap = 1.0;
    bool okp = false;
    for (int t = 0; t < kMaxTrials && !okp; ++t) {
      if (row)
        for (int j = 0; j < N; ++j) s.B[i * LD + j] = s.X[i * LD + j] + ap * s.A[i * LD + j];
      __syncthreads();
      okp = chol<LD, (kThreads<NP> > 64)>(s.B, N, &s.ok);
      if (!okp) ap *= 0.8;
    }
    real ad = 1.0;
    bool okd = false;
    for (int t = 0; t < kMaxTrials && !okd; ++t) {
      if (row)
        for (int j = 0; j < N; ++j)
          s.B[i * LD + j] = s.C[i * LD + j] - (i == j ? yi + ad * dyi : 0.0);
      __syncthreads();
      okd = chol<LD, (kThreads<NP> > 64)>(s.B, N, &s.ok);
      if (!okd) ad *= 0.8;
    }
    if (!okp && !okd) break;
    ap = okp ? ap * kStepFraction : 0.0;
    ad = okd ? ad * kStepFraction : 0.0;
    const real step = fmin(ap, ad);
    sigma = fmin(kSigmaMax, fmax(kSigmaMin, (1.0 - step) * (1.0 - step)));
    if (row) {
      for (int j = 0; j < N; ++j) s.X[i * LD + j] += ap * s.A[i * LD + j];
      yi += ad * dyi;
    }
    __syncthreads();
  }

  // leading eigenvector: X^32 (trace-normalised), then power iteration on
  // it from the last column of X
  square_normalised<NP, LD>(s.X, s.A, N, s.red);
  for (int q = 1; q < kSquarings; ++q)
    square_normalised<NP, LD>(q & 1 ? s.A : s.B, q & 1 ? s.B : s.A, N, s.red);
  const real* P = (kSquarings & 1) ? s.A : s.B;
  real u = row ? s.X[i * LD + N - 1] : 0.0;
  for (int p = 0; p < kPowerIters; ++p) {
    if (row) s.v[i] = u;
    __syncthreads();
    real w = 0.0;
    if (row)
      for (int j = 0; j < N; ++j) w += P[i * LD + j] * s.v[j];
    const real nrm = block_sum<NP>(w * w, s.red);
    u = nrm > 0.0 && isfinite(nrm) ? w / sqrt(nrm) : u;
    __syncthreads();
  }
  if (row) s.v[i] = u;
  __syncthreads();
  const real orient = s.v[N - 1] < 0.0 ? -1.0 : 1.0;  // the fixed entry of s~ non-negative
  if (i < N - 1) a.sbar[vec * (long long)(N - 1) + i] = skip || orient * u >= 0.0 ? 1 : -1;
  // primal Tr(C X) and, as diag(X) = 1, the duality gap <X, Z> = Tr(C X) - sum(y)
  real cx = 0.0;
  if (row)
    for (int j = 0; j < N; ++j) cx += s.X[i * LD + j] * s.C[i * LD + j];
  cx = block_sum<NP>(cx, s.red);
  const real ysum = block_sum<NP>(row ? yi : 0.0, s.red);
  if (i == 0) {
    if (a.objective) a.objective[vec] = run ? cx * scale : 0.0;
    if (a.gap) a.gap[vec] = run ? (cx - ysum) * scale : 0.0;
    if (a.iterations) a.iterations[vec] = it;
  }
  if (a.X && row)
    for (int j = 0; j < N; ++j) a.X[vec * (long long)N * N + (long long)i * N + j] = s.X[i * LD + j];
}

}  // namespace

hipError_t launch_sdr(const SdrArgs& a, hipStream_t s) {
  if (a.N <= 33)
    hipLaunchKernelGGL(sdr_kernel<33>, dim3(a.V), dim3(kThreads<33>), 0, s, a);
  else if (a.N <= 64)
    hipLaunchKernelGGL(sdr_kernel<64>, dim3(a.V), dim3(kThreads<64>), 0, s, a);
  else
    hipLaunchKernelGGL(sdr_kernel<65>, dim3(a.V), dim3(kThreads<65>), 0, s, a);
  return hipGetLastError();
}

}  // namespace taser
