// ||T~||_2 by Lanczos, shared by the preprocessing kernels of libtaser.so
// (Section III-C's step size tau = alpha / ||T~||_2).
#pragma once

#include "taser_internal.h"

namespace taser {
namespace spectral {

// Lanczos steps for ||T~||_2 to float32 resolution, from the start T~ e_N
// (alone, or with the small unstructured part that lanczos_norm adds).
// In the real form of a complex problem (QPSK) T~ borders a matrix whose
// eigenvalues come in pairs, and the Krylov space of T~ e_N stays in an
// invariant subspace of dimension (N + 1) / 2, so it needs about half the
// steps of a real problem (BPSK) of the same N.  The worst vector over B/U
// from 1/2 to 8 and SNR from -4 to 12 dB reached 1e-6 after 9, 15, 17, 20,
// 25, 27 and 30 steps for BPSK at N = 9, 17, 33, 49, 65, 97 and 129, and
// after 13, 12, 14, 16, 21 and 21 for QPSK at N = 17, 33, 49, 65, 97 and
// 129; the rule leaves a margin of three steps or more over those.
__host__ __device__ constexpr int lanczos_steps(int n, bool paired) {
  const int m = paired ? 12 + n / 8 : 16 + n / 4;
  return m < n ? m : n;
}
// the most steps any problem size of the library takes
constexpr int kLanczosMax = lanczos_steps(TASER_MAX_N, false);

// Sum over the 64 lanes of a wave, on the vector ALUs: rotations inside each
// 16-lane row (DPP row_ror 8, 4, 2, 1), then the gfx950 lane swaps across
// rows (permlane32 / permlane16: with both operands equal the two results
// are a value and its partner's).  A shuffle-based reduction goes through
// the LDS pipe, and the Lanczos reorthogonalisation makes hundreds of these
// reductions one after another.
__device__ __forceinline__ float wave_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x124, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x122, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x121, 0xF, 0xF, false));
  const unsigned u = __float_as_uint(v);
  const auto h = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  v = __uint_as_float(h[0]) + __uint_as_float(h[1]);
  const unsigned w = __float_as_uint(v);
  const auto r = __builtin_amdgcn_permlane16_swap(w, w, false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Sum over the four lanes n, n + 16, n + 32, n + 48 (the same position in the
// four 16-lane rows), by the two gfx950 lane swaps alone.
__device__ __forceinline__ float rows_sum(float v) {
  const unsigned u = __float_as_uint(v);
  const auto h = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  v = __uint_as_float(h[0]) + __uint_as_float(h[1]);
  const unsigned w = __float_as_uint(v);
  const auto r = __builtin_amdgcn_permlane16_swap(w, w, false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Hardware reciprocal, square root and reciprocal square root (about one
// ulp; the correctly rounded library forms cost some twenty instructions).
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float hsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Sturm count: number of eigenvalues of the symmetric tridiagonal
// (a[0..m-1], b[0..m-2]) that are smaller than x.
__device__ inline int sturm_count(const float* a, const float* b2, int m, float x, float pivmin) {
  int cnt = 0;
  float d = a[0] - x;
  if (fabsf(d) < pivmin) d = -pivmin;
  cnt += d < 0.f;
  for (int i = 1; i < m; ++i) {
    d = a[i] - x - b2[i - 1] * rcp(d);
    if (fabsf(d) < pivmin) d = -pivmin;
    cnt += d < 0.f;
  }
  return cnt;
}

// Largest (want_max) or smallest eigenvalue of a tridiagonal by 65-way
// multisection: each of the 64 lanes evaluates one interior point per round.
__device__ inline float tridiag_extreme(const float* a, const float* b2, int m, float lo, float hi,
                                 bool want_max, float pivmin) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int round = 0; round < 6; ++round) {
    const float w = (hi - lo) * (1.f / 65.f);
    const float x = lo + w * (float)(lane + 1);
    const int c = sturm_count(a, b2, m, x, pivmin);
    // want_max: first point with every eigenvalue below it bounds lambda_max
    // from above; want_min: first point with at least one eigenvalue below.
    const bool hit = want_max ? (c >= m) : (c >= 1);
    const unsigned long long mask = __ballot(hit);
    const int first = mask ? __ffsll((long long)mask) - 1 : kWave;
    const float new_hi = (first < kWave) ? lo + w * (float)(first + 1) : hi;
    const float new_lo = lo + w * (float)first;
    lo = new_lo;
    hi = new_hi;
    // a bracket within 1e-7 of the value is below the Lanczos resolution
    if (!(hi - lo > 1e-7f * fmaxf(fabsf(lo), fabsf(hi)))) break;
  }
  return 0.5f * (lo + hi);
}

// Deterministic Lanczos start vector with no structural zero component.
__device__ inline float start_entry(int i) {
  unsigned h = (unsigned)(i + 1) * 0x9E3779B9u;
  h ^= h >> 15;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  return 1.0f + (float)(h & 0xFFFFu) * (1.0f / 65536.0f);
}

// LDS floats lanczos_norm needs beside the basis: w (N) and the
// coefficients of one reorthogonalisation pass (one per basis vector).
__host__ __device__ constexpr int lanczos_scratch_floats(int n) { return n + kLanczosMax; }

// ||T~||_2 (largest |eigenvalue|) of the symmetric N x N matrix T, row-major
// in LDS, by Lanczos with full reorthogonalisation and a multisection of the
// Ritz tridiagonal.  The reorthogonalisation is classical Gram-Schmidt taken
// twice: each pass forms all coefficients q_i . w at once (four lanes per
// coefficient, one quarter of the rows each, met by two lane swaps) and then
// subtracts them together, so a pass waits on one reduction instead of one
// per basis vector.  Run by all 64 lanes of one wave (N <= 3 * 64); it takes
// lanczos_steps(N, paired) steps (paired: the real form of a complex
// problem); Q: LDS scratch of that many times N floats, al / be2: LDS arrays
// of as many floats, S: LDS scratch of lanczos_scratch_floats(N) floats.  T~ is
// semidefinite (coherent detection: T = A^T A; joint detection: T = -A^T A),
// so ||T~||_2 is its largest eigenvalue, or with nsd the magnitude of its
// smallest, and only that end of the spectrum is located.  Every lane
// returns the value.
__device__ inline float lanczos_norm(const float* T, int N, bool paired, bool nsd, float* Q,
                                     float* al, float* be2, float* S) {
  const int lane = threadIdx.x & (kWave - 1);
  const int m_cap = lanczos_steps(N, paired);
  // Start: the last column of T~ (the dominant eigenvector weighs the last
  // coordinate heavily, so few steps reach float32 resolution) plus 1 % of
  // a vector without structural zeros, so that an eigenvector orthogonal
  // to that column is still in the Krylov space.  Each lane reads and
  // writes only its own entries of Q.
  float nc = 0.f, ns = 0.f;
  for (int r = lane; r < N; r += kWave) {
    const float c = T[(size_t)r * N + N - 1], s = start_entry(r);
    nc += c * c;
    ns += s * s;
  }
  nc = wave_sum(nc);
  ns = wave_sum(ns);
  const float ic = nc > 0.f ? rsq(nc) : 0.f, is = 1e-2f * rsq(ns);
  float nrm = 0.f;
  for (int r = lane; r < N; r += kWave) {
    const float q = T[(size_t)r * N + N - 1] * ic + start_entry(r) * is;
    Q[r] = q;
    nrm += q * q;
  }
  nrm = wave_sum(nrm);
  const float inv0 = rsq(nrm);
  for (int r = lane; r < N; r += kWave) Q[r] *= inv0;
  int m = 0;
  float scale = 0.f;
  for (int j = 0; j < m_cap; ++j) {
    const float* q = Q + (size_t)j * N;
    float w[3];
    float dot = 0.f;
    for (int s = 0; s < 3; ++s) {
      const int r = lane + s * kWave;
      float acc = 0.f;
      if (r < N) {
        // four independent partial sums so that the LDS loads of the row
        // and of q pipeline instead of waiting one FMA at a time
        const float* row = T + (size_t)r * N;
        float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
        int k = 0;
        for (; k + 4 <= N; k += 4) {
          p0 += row[k] * q[k];
          p1 += row[k + 1] * q[k + 1];
          p2 += row[k + 2] * q[k + 2];
          p3 += row[k + 3] * q[k + 3];
        }
        for (; k < N; ++k) p0 += row[k] * q[k];
        acc = (p0 + p1) + (p2 + p3);
        dot += acc * q[r];
      }
      w[s] = acc;
    }
    const float alpha_j = wave_sum(dot);
    if (lane == 0) al[j] = alpha_j;
    m = j + 1;
    scale = fmaxf(scale, fabsf(alpha_j));
    if (j == m_cap - 1) break;
    // two passes of classical Gram-Schmidt against every Lanczos vector
    float* W = S;
    float* C = S + N;
    const int slice = lane >> 4;                  // quarter of the rows
    const int len = (N + 3) >> 2;
    const int r0 = slice * len, r1 = r0 + len < N ? r0 + len : N;
    for (int pass = 0; pass < 2; ++pass) {
      for (int s = 0; s < 3; ++s) { const int r = lane + s * kWave; if (r < N) W[r] = w[s]; }
      __builtin_amdgcn_wave_barrier();
      for (int base = 0; base <= j; base += 16) {
        const int i = base + (lane & 15);
        float p0 = 0.f, p1 = 0.f;
        if (i <= j) {
          const float* qi = Q + (size_t)i * N;
          int r = r0;
          for (; r + 2 <= r1; r += 2) {
            p0 = fmaf(qi[r], W[r], p0);
            p1 = fmaf(qi[r + 1], W[r + 1], p1);
          }
          if (r < r1) p0 = fmaf(qi[r], W[r], p0);
        }
        const float c = rows_sum(p0 + p1);
        if (slice == 0 && i <= j) C[i] = c;
      }
      __builtin_amdgcn_wave_barrier();
      for (int s = 0; s < 3; ++s) {
        const int r = lane + s * kWave;
        if (r < N) {
          float a0 = 0.f, a1 = 0.f;
          int i = 0;
          for (; i + 2 <= j + 1; i += 2) {
            a0 = fmaf(C[i], Q[(size_t)i * N + r], a0);
            a1 = fmaf(C[i + 1], Q[(size_t)(i + 1) * N + r], a1);
          }
          if (i <= j) a0 = fmaf(C[i], Q[(size_t)i * N + r], a0);
          w[s] -= a0 + a1;
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
    float bb = 0.f;
    for (int s = 0; s < 3; ++s) { const int r = lane + s * kWave; if (r < N) bb += w[s] * w[s]; }
    bb = wave_sum(bb);
    const float ib = bb > 0.f ? rsq(bb) : 0.f;
    const float beta = bb * ib;          // sqrt(bb)
    scale = fmaxf(scale, beta);
    if (!(beta > 1e-6f * scale)) break;   // invariant subspace found
    if (lane == 0) be2[j] = bb;
    float* qn = Q + (size_t)(j + 1) * N;
    for (int s = 0; s < 3; ++s) { const int r = lane + s * kWave; if (r < N) qn[r] = w[s] * ib; }
    __builtin_amdgcn_wave_barrier();
  }
  __builtin_amdgcn_wave_barrier();
  // Gershgorin interval of the Ritz tridiagonal
  float lo = 3.4e38f, hi = -3.4e38f;
  for (int i = 0; i < m; ++i) {
    const float r = (i > 0 ? hsqrt(be2[i - 1]) : 0.f) + (i < m - 1 ? hsqrt(be2[i]) : 0.f);
    lo = fminf(lo, al[i] - r);
    hi = fmaxf(hi, al[i] + r);
  }
  const float pivmin = 1e-30f + 1e-12f * fmaxf(fabsf(lo), fabsf(hi));
  return fabsf(tridiag_extreme(al, be2, m, lo, hi, !nsd, pivmin));
}

}  // namespace spectral
}  // namespace taser
