// Reference detectors of the paper's comparison (Section V-A): the matched
// filter (Algorithm 1's one-iteration limit), linear MMSE, exhaustive ML and
// K-best tree search, on the real-valued model of Section II-A
// (ybar = Hbar sbar + nbar, sbar in {-1,+1}^M, M = N - 1).
//
// One wave per vector.  It forms the complex Gram G = H^H H and b = H^H y,
// writes the real form A = Hbar^T Hbar ([[Re G, -Im G], [Im G, Re G]] for
// QPSK, Re G for BPSK) and bbar = Hbar^T ybar to LDS, then:
//   MF     signs of bbar;
//   MMSE   (A + (N0/2) I) x = bbar by an in-LDS Cholesky factorisation
//          (lane i owns row i) and two triangular solves;
//   ML     all 2^M candidates, lane l taking those whose top bits are l, in
//          Gray-code order: flipping s_k changes f(s) = s^T A s - 2 bbar^T s
//          by 4 (A_kk - s_k (r_k - bbar_k)) with r = A s, and r moves by
//          -2 s_k A_:k; r and f are recomputed from scratch every 256
//          candidates so that float32 rounding does not accumulate;
//   K-best Cholesky A = L L^T gives R = L^T and z = L^-1 bbar with
//          ||ybar - Hbar s||^2 = ||z - R s||^2 + ||ybar||^2 - ||z||^2; from
//          the last real dimension to the first every surviving path is
//          extended by +1 and -1 (one lane per candidate) and the K of
//          smallest partial distance survive, ranked by counting (ties: the
//          earlier candidate, path rank first, +1 before -1).
#include <math.h>

#include "taser_internal.h"

namespace taser {
namespace {

constexpr int kMaxM = 64;          // real dimensions (U <= 32 QPSK, U <= 64 BPSK)
constexpr int kLd = kMaxM + 1;     // LDS row stride of A
constexpr int kMaxK = 16;          // K-best survivors (2K candidates <= 32 lanes)
constexpr int kMaxMl = 20;         // exhaustive ML: 2^20 candidates at most

struct RefLds {
  float A[kMaxM * kLd];            // Hbar^T Hbar, then its Cholesky factor
  float b[kMaxM];                  // Hbar^T ybar, then z or x
  float yy;                        // ||y||^2
  float pd[2][kMaxK];              // K-best partial distances (double buffered)
  float cand[2 * kMaxK];
  signed char sym[2][kMaxK][kMaxM];
};

__device__ __forceinline__ float2 cmul_conj(float2 a, float2 b) {   // conj(a) b
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// A = Hbar^T Hbar, b = Hbar^T ybar, yy = ||y||^2 into LDS.
__device__ void build_normal(const RefArgs& a, long long v, RefLds& s) {
  const int lane = threadIdx.x;
  const int B = a.B, U = a.U;
  const bool qpsk = a.mod == TASER_QPSK;
  const float2* H = a.H + (v / a.y_per_H) * (long long)B * U;
  const float2* y = a.y + v * (long long)B;
  // Hermitian G: entries (u1 <= u2), lane-strided
  for (int e = lane; e < U * U; e += 64) {
    const int u1 = e / U, u2 = e % U;
    if (u1 > u2) continue;
    float re = 0.f, im = 0.f;
    for (int r = 0; r < B; ++r) {
      const float2 p = cmul_conj(H[(long long)r * U + u1], H[(long long)r * U + u2]);
      re += p.x;
      im += p.y;
    }
    // real form: [[Re G, -Im G], [Im G, Re G]] (QPSK) or Re G (BPSK)
    s.A[u1 * kLd + u2] = re;
    s.A[u2 * kLd + u1] = re;
    if (qpsk) {
      s.A[(U + u1) * kLd + U + u2] = re;
      s.A[(U + u2) * kLd + U + u1] = re;
      s.A[u1 * kLd + U + u2] = -im;       // -Im G_{u1 u2}
      s.A[(U + u2) * kLd + u1] = -im;
      s.A[(U + u1) * kLd + u2] = im;      // Im G_{u1 u2}
      s.A[u2 * kLd + U + u1] = im;
    }
  }
  for (int u = lane; u < U; u += 64) {
    float re = 0.f, im = 0.f;
    for (int r = 0; r < B; ++r) {
      const float2 p = cmul_conj(H[(long long)r * U + u], y[r]);
      re += p.x;
      im += p.y;
    }
    s.b[u] = re;
    if (qpsk) s.b[U + u] = im;
  }
  float yy = 0.f;
  for (int r = lane; r < B; r += 64) yy += y[r].x * y[r].x + y[r].y * y[r].y;
  for (int o = 32; o > 0; o >>= 1) yy += __shfl_xor(yy, o, 64);
  if (lane == 0) s.yy = yy;
  __syncthreads();
}

// In-place Cholesky A = L L^T of the leading M x M block (lane i owns row i);
// a non-positive pivot (a singular or indefinite matrix) is replaced by the
// smallest normal float so that the arithmetic stays finite.
__device__ void cholesky(RefLds& s, int M) {
  const int i = threadIdx.x;
  for (int k = 0; k < M; ++k) {
    if (i == k) {
      const float d = s.A[k * kLd + k];
      s.A[k * kLd + k] = d > 0.f ? sqrtf(d) : 1.17549435e-38f;
    }
    __syncthreads();
    if (i > k && i < M) s.A[i * kLd + k] /= s.A[k * kLd + k];
    __syncthreads();
    if (i > k && i < M) {
      const float lik = s.A[i * kLd + k];
      for (int j = k + 1; j <= i; ++j) s.A[i * kLd + j] -= lik * s.A[j * kLd + k];
    }
    __syncthreads();
  }
}

// z = L^-1 b in place.
__device__ void forward_solve(RefLds& s, int M) {
  const int i = threadIdx.x;
  for (int k = 0; k < M; ++k) {
    if (i == k) s.b[k] /= s.A[k * kLd + k];
    __syncthreads();
    if (i > k && i < M) s.b[i] -= s.A[i * kLd + k] * s.b[k];
    __syncthreads();
  }
}

// x = L^-T z in place.
__device__ void backward_solve(RefLds& s, int M) {
  const int i = threadIdx.x;
  for (int k = M - 1; k >= 0; --k) {
    if (i == k) s.b[k] /= s.A[k * kLd + k];
    __syncthreads();
    if (i < k) s.b[i] -= s.A[k * kLd + i] * s.b[k];
    __syncthreads();
  }
}

__global__ __launch_bounds__(64) void ref_linear_kernel(RefArgs a) {
  __shared__ RefLds s;
  const long long v = blockIdx.x;
  const int M = a.M;
  build_normal(a, v, s);
  if (a.kind == TASER_REF_MMSE) {
    const int i = threadIdx.x;
    if (i < M) s.A[i * kLd + i] += 0.5f * a.n0;
    __syncthreads();
    cholesky(s, M);
    forward_solve(s, M);
    backward_solve(s, M);
  }
  for (int k = threadIdx.x; k < M; k += 64) {
    const float x = s.b[k];
    a.sbar[v * M + k] = x >= 0.f ? 1 : -1;
    if (a.soft) a.soft[v * M + k] = x;
  }
}

__global__ __launch_bounds__(64) void ref_kbest_kernel(RefArgs a) {
  __shared__ RefLds s;
  const long long v = blockIdx.x;
  const int M = a.M, K = a.K;
  const int lane = threadIdx.x;
  build_normal(a, v, s);
  cholesky(s, M);
  forward_solve(s, M);                     // b <- z
  // partial distance of path p through level i uses R_im = L_mi (m >= i)
  int np = 1, cur = 0;
  if (lane == 0) s.pd[0][0] = 0.f;
  __syncthreads();
  for (int i = M - 1; i >= 0; --i) {
    const int nc = 2 * np;
    float pd = 3.4e38f;
    const int p = lane >> 1;
    const float sym = (lane & 1) ? -1.f : 1.f;
    if (lane < nc) {
      float e = s.b[i] - s.A[i * kLd + i] * sym;
      for (int m = i + 1; m < M; ++m) e -= s.A[m * kLd + i] * (float)s.sym[cur][p][m];
      pd = s.pd[cur][p] + e * e;
      s.cand[lane] = pd;
    }
    __syncthreads();
    if (lane < nc) {
      int rank = 0;
      for (int c = 0; c < nc; ++c) {
        const float q = s.cand[c];
        rank += (q < pd || (q == pd && c < lane)) ? 1 : 0;
      }
      if (rank < K) {
        const int nxt = cur ^ 1;
        for (int m = i + 1; m < M; ++m) s.sym[nxt][rank][m] = s.sym[cur][p][m];
        s.sym[nxt][rank][i] = (signed char)sym;
        s.pd[nxt][rank] = pd;
      }
    }
    __syncthreads();
    cur ^= 1;
    np = nc < K ? nc : K;
  }
  for (int k = lane; k < M; k += 64) a.sbar[v * M + k] = s.sym[cur][0][k];
  if (a.soft && lane == 0) {
    float zz = 0.f;
    for (int k = 0; k < M; ++k) zz += s.b[k] * s.b[k];
    a.soft[v] = s.pd[cur][0] + (s.yy - zz);
  }
}

// f(s) = s^T A s - 2 b^T s for the candidate with bit pattern `bits`
// (bit j set: s_j = -1), and r = A s.
__device__ __forceinline__ float ml_start(const RefLds& s, int M, unsigned bits, float (&r)[kMaxMl]) {
  float f = 0.f;
#pragma unroll
  for (int k = 0; k < kMaxMl; ++k) {
    if (k >= M) { r[k] = 0.f; continue; }
    float acc = 0.f;
    for (int j = 0; j < M; ++j) acc += s.A[k * kLd + j] * (((bits >> j) & 1u) ? -1.f : 1.f);
    r[k] = acc;
    const float sk = ((bits >> k) & 1u) ? -1.f : 1.f;
    f += sk * (acc - 2.f * s.b[k]);
  }
  return f;
}

__global__ __launch_bounds__(64) void ref_ml_kernel(RefArgs a) {
  __shared__ RefLds s;
  const long long v = blockIdx.x;
  const int M = a.M;
  const int lane = threadIdx.x;
  build_normal(a, v, s);
  // lane l takes the candidates whose top hb bits are l
  const int hb = M < 6 ? M : 6;
  const int lo = M - hb;                    // bits enumerated inside a lane
  const int gb = lo < 8 ? lo : 8;           // Gray-code bits per block (r, f recomputed per block)
  const int blocks = 1 << (lo - gb);
  float best = 3.4e38f;
  unsigned best_bits = 0;
  if (lane < (1 << hb)) {
    float r[kMaxMl];
    for (int blk = 0; blk < blocks; ++blk) {
      unsigned bits = ((unsigned)lane << lo) | ((unsigned)blk << gb);
      float f = ml_start(s, M, bits, r);
      if (f < best) { best = f; best_bits = bits; }
      for (unsigned t = 1; t < (1u << gb); ++t) {
        const int k = __builtin_ctz(t);      // the same in every lane
        const float sk = ((bits >> k) & 1u) ? -1.f : 1.f;
        float rk = 0.f;
#pragma unroll
        for (int j = 0; j < kMaxMl; ++j) rk = j == k ? r[j] : rk;
        f += 4.f * (s.A[k * kLd + k] - sk * (rk - s.b[k]));
        const float m2s = -2.f * sk;
#pragma unroll
        for (int j = 0; j < kMaxMl; ++j)
          if (j < M) r[j] = fmaf(m2s, s.A[j * kLd + k], r[j]);
        bits ^= 1u << k;
        if (f < best || (f == best && bits < best_bits)) { best = f; best_bits = bits; }
      }
    }
  }
  // wave argmin (ties: the smaller bit pattern)
  for (int o = 32; o > 0; o >>= 1) {
    const float ob = __shfl_xor(best, o, 64);
    const unsigned obits = (unsigned)__shfl_xor((int)best_bits, o, 64);
    if (ob < best || (ob == best && obits < best_bits)) { best = ob; best_bits = obits; }
  }
  for (int k = lane; k < M; k += 64) a.sbar[v * M + k] = ((best_bits >> k) & 1u) ? -1 : 1;
  if (a.soft && lane == 0) a.soft[v] = best + s.yy;
}

}  // namespace

hipError_t launch_reference(const RefArgs& a, hipStream_t s) {
  const dim3 grid(a.V), block(64);
  if (a.kind == TASER_REF_KBEST)
    hipLaunchKernelGGL(ref_kbest_kernel, grid, block, 0, s, a);
  else if (a.kind == TASER_REF_ML)
    hipLaunchKernelGGL(ref_ml_kernel, grid, block, 0, s, a);
  else
    hipLaunchKernelGGL(ref_linear_kernel, grid, block, 0, s, a);
  return hipGetLastError();
}

}  // namespace taser
