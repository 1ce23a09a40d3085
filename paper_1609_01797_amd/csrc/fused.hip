// Fused single-launch TASER for groups of 16 received vectors that share
// one channel matrix H (coherent QPSK, U = 16 users, N = 33).
//
// One wave detects one group.  The 16 vectors are the N dimension of
// 16x16x4 float32 MFMAs, so the preconditioned Gram block G~ (the 32x32
// upper-left block of T~, identical for the 16 vectors) is the shared A
// operand and stays in 16 VGPRs for the whole solve.  T~ is bordered:
//     T~ = [ G~    c~_v ]      L~ = [ L11   0   ]
//          [ c~_v^T  1  ]           [ l21^T l22 ]
// Row i of V = L~ - tril(2 tau L~ T~) (the gradient step of Algorithm 1)
// depends on row i of L~ only, so the rows are processed one after another in
// registers.  Register layout: lane l serves vector n = l % 16 and column
// quad g = l / 16; for a row of L~ it holds columns 16 mt + 4 r + g
// (mt in {0,1}, r in 0..3) in register (mt, r).  With the MFMA output rows
// permuted by jj(m) = 4 (m % 4) + m / 4, the product's output registers are
// exactly the next iteration's B operands, and each K-step covers four
// consecutive columns, so the triangular structure skips whole K-steps.
// Column norms (the prox of Section III-C) are then sums inside a lane.
#include <math.h>

#include <type_traits>

#include "taser_internal.h"

namespace taser {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

template <int Begin, int End, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (Begin < End) {
    f(std::integral_constant<int, Begin>{});
    sfor<Begin + 1, End>(f);
  }
}

__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Sum over the four lanes that serve one vector (lanes n, n+16, n+32, n+48)
// with the gfx950 lane-swap instructions (no LDS round trip).  With both
// operands equal, the two results of a swap hold x and its partner's x in
// every lane, so their sum is the pairwise sum: first across the two 32-lane
// halves, then across adjacent 16-lane rows.
__device__ __forceinline__ float sum_groups(float x) {
  const unsigned u = __float_as_uint(x);
  const auto h = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  const float y = __uint_as_float(h[0]) + __uint_as_float(h[1]);
  const unsigned w = __float_as_uint(y);
  const auto r = __builtin_amdgcn_permlane16_swap(w, w, false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ int or_groups(int x) {
  const auto h = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)x, false, false);
  const unsigned y = h[0] | h[1];
  const auto r = __builtin_amdgcn_permlane16_swap(y, y, false, false);
  return (int)(r[0] | r[1]);
}

// Hardware reciprocal, square root and reciprocal square root (about one
// ulp; the correctly rounded library forms cost some twenty instructions).
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float hsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// 16-bit operands for the BF16 / FP16 products: four values packed in two
// dwords, element e holding MFMA K position 4 (lane / 16) + e.
typedef unsigned u2 __attribute__((ext_vector_type(2)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));

// Two float32 values to packed 16-bit (round to nearest even): one
// v_cvt_pk_bf16_f32 / v_cvt_pk_f16_f32, visible to the compiler's hazard
// tracking (the conversion feeds an MFMA source directly).
template <int P>
__device__ __forceinline__ unsigned cvt_pk(float lo, float hi) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  const f2 x = {lo, hi};
  if constexpr (P == TASER_PREC_BF16) {
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(unsigned, __builtin_convertvector(x, b2));
  } else {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(unsigned, __builtin_convertvector(x, h2));
  }
}

template <int P>
__device__ __forceinline__ u2 pack4(float x0, float x1, float x2, float x3) {
  return u2{cvt_pk<P>(x0, x1), cvt_pk<P>(x2, x3)};
}

template <int P>
__device__ __forceinline__ f4 mfma16(u2 a, u2 b, f4 c) {
  if constexpr (P == TASER_PREC_BF16)
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a),
                                                     __builtin_bit_cast(s4, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(h4, a),
                                                 __builtin_bit_cast(h4, b), c, 0, 0, 0);
}

// One 16x16x32 product: the K slots of the two 16-column tiles (kt = 0, 1)
// side by side, a = [a0, a1], b = [b0, b1].  On gfx950 it takes the cycles of
// one 16x16x16 product for twice the work.
typedef unsigned u4 __attribute__((ext_vector_type(4)));
template <int P>
__device__ __forceinline__ f4 mfma32(u2 a0, u2 a1, u2 b0, u2 b1, f4 c) {
  const u4 a = {a0[0], a0[1], a1[0], a1[1]}, b = {b0[0], b0[1], b1[0], b1[1]};
  if constexpr (P == TASER_PREC_BF16) {
    typedef __bf16 b8 __attribute__((ext_vector_type(8)));
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, a),
                                                   __builtin_bit_cast(b8, b), c, 0, 0, 0);
  } else {
    typedef _Float16 h8v __attribute__((ext_vector_type(8)));
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8v, a),
                                                  __builtin_bit_cast(h8v, b), c, 0, 0, 0);
  }
}

// Krylov dimension for ||T~||_2.  Twelve steps of the plain float32
// recurrence from [c~; 1] bring the top Ritz value within 1e-6 of ||T~||_2 on
// 128x16 channels from 0 dB up; at -4 dB about one vector in 4,000 is still
// 2e-5 below it (its top eigenvalue is less dominant).  One or two more steps
// would close that but produce ghost copies of the converged Ritz value (loss
// of orthogonality), which slow Laguerre's method to linear convergence and
// cost more than the steps themselves.
constexpr int kLanczosSteps = 12;
constexpr int kLaguerreIters = 8;

// Largest eigenvalue of the symmetric tridiagonal (al, b2 = beta^2) of size M
// by Laguerre's method from the Gershgorin upper bound.  The characteristic
// polynomial has only real roots, so from the right the iteration decreases
// monotonically to the largest root (cubic convergence).  The ratios
// d_k = p_k / p_{k-1} of the leading principal minors of (x I - T) give
// G = p'/p and H = -(p'/p)'.
template <int M>
__device__ __forceinline__ float tridiag_top(const float (&al)[M], const float (&b2)[M]) {
  float x = -3.4e38f;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const float rad = (k > 0 ? hsqrt(b2[k - 1]) : 0.f) + (k < M - 1 ? hsqrt(b2[k]) : 0.f);
    x = fmaxf(x, al[k] + rad);
  }
  x = x * (1.f + 1e-6f) + 1e-30f;
  for (int it = 0; it < kLaguerreIters; ++it) {
    float d = x - al[0];
    float e = 1.f, f = 0.f;
    float id = rcp(d);
    float G = e * id, Hs = G * G;
#pragma unroll
    for (int k = 1; k < M; ++k) {
      const float dn = (x - al[k]) - b2[k - 1] * id;
      const float en = 1.f + b2[k - 1] * e * id * id;
      const float fn = b2[k - 1] * id * id * (f - 2.f * e * e * id);
      d = dn; e = en; f = fn;
      id = rcp(d);
      const float r = e * id;
      G += r;
      Hs += r * r - f * id;
    }
    const float disc = fmaxf(0.f, (float)(M - 1) * ((float)M * Hs - G * G));
    const float step = (float)M * rcp(G + hsqrt(disc));
    if (!(step > 0.f) || !isfinite(step)) break;
    x -= step;
    // cubic convergence: once a step is this small the next one would be
    // below float32 resolution
    if (step <= 1e-5f * x) break;
  }
  return x;
}

// Workspace per channel group (floats): the MFMA A operands of G~ (its real
// and imaginary parts R and M; the real form [[R, -M], [M, R]] is rebuilt in
// registers) and the border c~, stored register-major ([register][lane]) so
// both kernels move them coalesced; then the 16 column scales D (column
// quad g and register r: entry 4 r + g), and D_NN, tau and flags per vector
// (entry n).  The state does not depend on the product precision, so one
// preparation can feed solves of every precision.
constexpr int kWsR = 0, kWsM = 256, kWsC = 512, kWsD = 1024, kWsDN = 1040, kWsTau = 1056,
              kWsFlag = 1072;
constexpr int kWsFloats = 1088;
static_assert(kWsFloats * sizeof(float) == kGroupWsBytes, "group workspace size");

// Waves (channel groups) per workgroup of the preparation kernel.  Its
// waves need few registers, so five would fit on a SIMD; four-wave
// workgroups put one wave on each SIMD of a CU, which keeps a batch of
// 4 x 1024 groups evenly spread (with one-wave workgroups some SIMDs took
// five groups and others three, and the kernel lasts as long as the fullest).
constexpr int kPrepWaves = 4;

// Preprocessing of one channel group (one wave): T~ in bordered form and the
// step size, stored to the workspace in the register layout of the solve.
// The complex Gram arrives as MFMA accumulators (lane (n, g) holds rows
// 4 g + r of column n): reG = Re G, imG = P = Hr^T Hi (Im G = P - P^T),
// reb / imb = Re / Im of b = H^H y, and the lane's part of ||y||^2.  Every
// wave of the workgroup calls it (the step size uses workgroup barriers);
// waves without a group (active false) compute on zeros and store nothing.
__device__ __forceinline__ void prep_finish(const FusedArgs& a, long long grp, bool active,
                                            const f4& reG, const f4& imG, const f4& reb,
                                            const f4& imb, float ysq) {
  // one LDS region per wave of the workgroup (each wave is one group)
  __shared__ float2 Gs_all[kPrepWaves][16 * 16];   // G = H^H H, [row][col]
  __shared__ float2 bs_all[kPrepWaves][16 * 16];   // b = H^H y, [user][vector]
  __shared__ float yy2_all[kPrepWaves][16];        // ||y||^2 per vector

  const int lane = threadIdx.x & 63;
  const int n = lane & 15;         // vector within the group (MFMA N index)
  const int g = lane >> 4;         // column quad (MFMA K / output row group)
  const long long v = grp * 16 + n;
  float2* Gs = Gs_all[threadIdx.x >> 6];
  float2* bs = bs_all[threadIdx.x >> 6];
  float* yy2 = yy2_all[threadIdx.x >> 6];

  ysq = sum_groups(ysq);
  // imG holds P = Hr^T Hi; Im G = P - P^T
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    Gs[(4 * g + r) * 16 + n] = make_float2(reG[r], imG[r]);
    bs[(4 * g + r) * 16 + n] = make_float2(reb[r], imb[r]);
  }
  if (g == 0) yy2[n] = ysq;
  // one wave: its LDS accesses complete in program order; the barriers keep
  // the compiler from moving LDS reads and writes across each other
  __builtin_amdgcn_wave_barrier();
  float pt[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) pt[r] = Gs[n * 16 + 4 * g + r].y;
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int r = 0; r < 4; ++r) Gs[(4 * g + r) * 16 + n].y = imG[r] - pt[r];
  __builtin_amdgcn_wave_barrier();

  // ---------------- Jacobi preconditioning (Section III-C) ----------------
  bool bad_group = false, deg_group = false, bad_vec = false, deg_vec = false;
  auto Du = [&](int u) {
    const float d = fabsf(Gs[u * 17].x);
    return d == 0.f ? 1.f : hsqrt(d);
  };
  const float yn = yy2[n];
  deg_vec = yn == 0.f;
  bad_vec = !isfinite(yn);
  const float DN = (yn == 0.f || !isfinite(yn)) ? 1.f : hsqrt(yn);

  // per-lane column data: columns j = 16 mt + 4 r + g, user u = 4 r + g
  float Dc[4], ct[2][4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int u = 4 * r + g;
    Dc[r] = Du(u);
    const float2 bu = bs[u * 16 + n];
    if (!isfinite(bu.x) || !isfinite(bu.y)) bad_vec = true;
    const float inv = rcp(Dc[r] * DN);
    ct[0][r] = -bu.x * inv;          // last column of T: -Hbar^T ybar
    ct[1][r] = -bu.y * inv;
  }
  // A operands: A[mt][kt][s] = G~[16 mt + jj(n)][16 kt + 4 s + g]; the
  // column user 4 s + g is the lane's user of Dc[s]
  float A[2][2][4];
  {
    const int aa = 4 * (n & 3) + (n >> 2);
    const float da = Du(aa);
    if (Gs[aa * 17].x == 0.f) deg_group = true;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int bb = 4 * s + g;
      const float2 gab = Gs[aa * 16 + bb];
      if (!isfinite(gab.x) || !isfinite(gab.y)) bad_group = true;
      const float inv = rcp(da * Dc[s]);
      A[0][0][s] = gab.x * inv;
      A[0][1][s] = -gab.y * inv;
      A[1][0][s] = gab.y * inv;
      A[1][1][s] = gab.x * inv;
    }
  }
  // group-wide and per-vector flags
  const unsigned long long mg = __ballot(bad_group) | 0ull;
  const unsigned long long md = __ballot(deg_group) | 0ull;
  const unsigned long long mbv = __ballot(bad_vec);
  const unsigned long long mdv = __ballot(deg_vec);
  auto fold = [&](unsigned long long m) {
    return (unsigned)((m | (m >> 16) | (m >> 32) | (m >> 48)) & 0xFFFFull);
  };
  const bool nonfinite = mg != 0ull || ((fold(mbv) >> n) & 1u);
  const bool degenerate = !nonfinite && (md != 0ull || ((fold(mdv) >> n) & 1u));
  const bool skip = nonfinite || degenerate;
  if (skip) {
    // keep the arithmetic of the other vectors clean; this vector's results
    // are replaced at the end
#pragma unroll
    for (int r = 0; r < 4; ++r) { ct[0][r] = 0.f; ct[1][r] = 0.f; }
  }
  if (mg != 0ull) {
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int kt = 0; kt < 2; ++kt)
#pragma unroll
        for (int s = 0; s < 4; ++s) A[mt][kt][s] = 0.f;
  }

  // ---------------- step size tau = alpha / ||T~||_2 ----------------
  float tau;
  if (a.tau_mode == TASER_TAU_GIVEN) {
    tau = active ? a.tau_in[v] : 1.f;
  } else {
    // Lanczos from T~ e_N = [c~; 1] (a good start: the dominant eigenvector of
    // T~ weighs the last coordinate heavily), plain three-term recurrence.
    // alpha_j and beta_j^2 go straight to LDS, where one wave of the
    // workgroup takes them for the eigenvalue step below; a rolled loop
    // keeps the kernel's code small.
    __shared__ float tri_all[kPrepWaves][2 * kLanczosSteps][16];   // al, then b2
    __shared__ float lam_all[kPrepWaves][16];
    const int w = threadIdx.x >> 6;
    float Q[2][4], Qp[2][4], q32, qp32 = 0.f, beta = 0.f;
    float nrm = 0.f;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) { Q[mt][r] = ct[mt][r]; Qp[mt][r] = 0.f; nrm += Q[mt][r] * Q[mt][r]; }
    nrm = sum_groups(nrm) + 1.f;
    const float inv0 = rsq(nrm);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) Q[mt][r] *= inv0;
    q32 = inv0;
    bool done = false;
    float scale = 0.f;
    // G~ = R + i M is Hermitian with real form [[R, -M], [M, R]] (the blocks
    // A[0][0] and A[1][0]), so G~ q for q = [c; d] takes three real products
    // instead of four (Gauss's complex product):
    //   k1 = (R + M) c,  k2 = R (d - c),  k3 = M (c + d),
    //   [R c - M d; M c + R d] = [k1 - k3; k1 + k2].
    float Apm[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) Apm[s] = A[0][0][s] + A[1][0][s];
#pragma unroll 2
    for (int j = 0; j < kLanczosSteps; ++j) {
      f4 k1 = {0.f, 0.f, 0.f, 0.f}, k2 = k1, k3 = k1;
      // issue priority while this wave feeds the matrix pipe (here and in the
      // Gram below): the four waves of a SIMD otherwise leave it idle while
      // they all run vector-ALU work
      __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        k1 = mfma(Apm[s], Q[0][s], k1);
        k2 = mfma(A[0][0][s], Q[1][s] - Q[0][s], k2);
        k3 = mfma(A[1][0][s], Q[0][s] + Q[1][s], k3);
      }
      __builtin_amdgcn_s_setprio(0);
      float W[2][4];
      float cq = 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        W[0][r] = (k1[r] - k3[r]) + ct[0][r] * q32;
        W[1][r] = (k1[r] + k2[r]) + ct[1][r] * q32;
      }
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) cq += ct[mt][r] * Q[mt][r];
      float w32 = sum_groups(cq) + q32;
      float dot = 0.f;
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) dot += W[mt][r] * Q[mt][r];
      const float alj = sum_groups(dot) + w32 * q32;
      float ww = 0.f;
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          W[mt][r] = fmaf(-alj, Q[mt][r], fmaf(-beta, Qp[mt][r], W[mt][r]));
          ww += W[mt][r] * W[mt][r];
        }
      w32 = fmaf(-alj, q32, fmaf(-beta, qp32, w32));
      const float bb = sum_groups(ww) + w32 * w32;
      // After a breakdown (an invariant Krylov subspace) the remaining
      // diagonal entries are parked far below the spectrum and decoupled.
      float alo = -1e30f, b2o = 0.f;
      if (!done) {
        alo = alj;
        b2o = bb;
        scale = fmaxf(scale, fabsf(alj));
        if (!(bb > 1e-12f * scale * scale)) { done = true; b2o = 0.f; }
      }
      if (g == 0) {
        tri_all[w][j][n] = alo;
        tri_all[w][kLanczosSteps + j][n] = b2o;
      }
      const float ib = bb > 0.f ? rsq(bb) : 0.f;
      beta = bb * ib;                 // sqrt(bb)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) { Qp[mt][r] = Q[mt][r]; Q[mt][r] = W[mt][r] * ib; }
      qp32 = q32;
      q32 = w32 * ib;
    }
    // The top eigenvalue of each tridiagonal is a serial recurrence per
    // vector, which the four lanes of a vector would repeat.  Instead one
    // wave of the workgroup takes all 64 vectors of its four groups, one per
    // lane (the wave chosen by the workgroup index, so that on a CU the work
    // spreads over the SIMDs).
    __syncthreads();
    if (w == (int)(blockIdx.x & (kPrepWaves - 1))) {
      float al2[kLanczosSteps], b22[kLanczosSteps];
#pragma unroll
      for (int k = 0; k < kLanczosSteps; ++k) {
        al2[k] = tri_all[lane >> 4][k][n];
        b22[k] = tri_all[lane >> 4][kLanczosSteps + k][n];
      }
      lam_all[lane >> 4][n] = tridiag_top<kLanczosSteps>(al2, b22);
    }
    __syncthreads();
    const float lam = lam_all[w][n];
    tau = a.alpha / (lam > 0.f ? lam : 1.f);
  }
  if (!active) return;
  // ---------------- hand the group's state to the solve kernel ----------------
  float* ws = a.ws + grp * kWsFloats;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    ws[kWsR + s * 64 + lane] = A[0][0][s];
    ws[kWsM + s * 64 + lane] = A[1][0][s];
  }
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) ws[kWsC + (mt * 4 + r) * 64 + lane] = ct[mt][r];
  // D depends on the column only, D_NN, tau and the flags on the vector only
  if (n == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) ws[kWsD + 4 * r + g] = Dc[r];
  }
  if (g == 0) {
    ws[kWsDN + n] = DN;
    ws[kWsTau + n] = tau;
    ws[kWsFlag + n] = __int_as_float((nonfinite ? 2 : 0) | (degenerate ? 1 : 0));
  }
  if (g == 0 && a.status)
    a.status[v] = nonfinite ? TASER_VEC_NONFINITE : (degenerate ? TASER_VEC_DEGENERATE : 0);
}


// One row-quad of the channel group: lane (n, g) holds H[4 q + g][n] and
// y_n[4 q + g]; six 16x16x4 MFMAs add its share of G and b.  Im G is not
// accumulated directly: with P = Hr^T Hi, Im G = P - P^T (formed once the
// sums are complete).  b = H^H y takes three real products (Gauss's complex
// product): k1 = (Hr - Hi)^T yr, k2 = Hr^T (yi - yr), k3 = Hi^T (yr + yi),
// Re b = k1 + k3, Im b = k1 + k2.
__device__ __forceinline__ void gram_rowquad(float2 h, float2 y, f4& reG, f4& pG, f4& k1,
                                             f4& k2, f4& k3, float& ysq) {
  reG = mfma(h.x, h.x, reG);       // Re G = Hr^T Hr + Hi^T Hi
  reG = mfma(h.y, h.y, reG);
  pG = mfma(h.x, h.y, pG);         // P = Hr^T Hi
  k1 = mfma(h.x - h.y, y.x, k1);
  k2 = mfma(h.x, y.y - y.x, k2);
  k3 = mfma(h.y, y.x + y.y, k3);
  ysq += y.x * y.x + y.y * y.y;
}

// Any B: rows are consumed in batches of 8 row-quads; the next batch's loads
// are issued before the current batch's MFMAs so that load latency overlaps.
__global__ __launch_bounds__(64 * kPrepWaves) void prep_group_qpsk16(FusedArgs a, int groups) {
  const int lane = threadIdx.x & 63;
  const int n = lane & 15;
  const int g = lane >> 4;
  const long long grp = (long long)blockIdx.x * kPrepWaves + (threadIdx.x >> 6);
  // waves past the last group stay for the workgroup barriers of the step size
  const bool active = grp < groups;
  const int B = active ? a.B : 0;
  const float2* Hg = a.H + (grp * 16 / a.y_per_H) * (long long)B * 16;
  const float2* yv = a.y + (grp * 16 + n) * B;
  f4 reG = {0.f, 0.f, 0.f, 0.f}, pG = reG, k1 = reG, k2 = reG, k3 = reG;
  float ysq = 0.f;
  constexpr int kQ = 8;
  float2 h0[kQ], y0[kQ], h1[kQ], y1[kQ];
  // Any assignment of a batch's rows to the (slot, lane) pairs gives the same
  // sums as long as h and y agree.  Whole batches (the common case) load
  // without per-row guards, from one base pointer with immediate offsets:
  // with B even, slot 2 p + e holds row r0 + 8 p + 2 g + e, so each lane
  // reads two consecutive entries of y in one 16-byte load; otherwise (and
  // in the last, partial batch) slot q holds row r0 + 4 q + g.
  auto load_batch = [&](int r0, float2 (&hb)[kQ], float2 (&yb)[kQ]) {
    if (r0 + 4 * kQ <= B && (B & 1) == 0) {
      const float2* hp = Hg + (long long)(r0 + 2 * g) * 16 + n;
      const float4* yp = reinterpret_cast<const float4*>(yv + r0 + 2 * g);
#pragma unroll
      for (int p = 0; p < kQ / 2; ++p) {
        const float4 t = yp[4 * p];
        yb[2 * p] = make_float2(t.x, t.y);
        yb[2 * p + 1] = make_float2(t.z, t.w);
        hb[2 * p] = hp[128 * p];
        hb[2 * p + 1] = hp[128 * p + 16];
      }
      return;
    }
    const float2* hp = Hg + (long long)(r0 + g) * 16 + n;
    const float2* yp = yv + r0 + g;
    if (r0 + 4 * kQ <= B) {
#pragma unroll
      for (int q = 0; q < kQ; ++q) { hb[q] = hp[64 * q]; yb[q] = yp[4 * q]; }
    } else {
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const bool in = r0 + 4 * q + g < B;
        hb[q] = in ? hp[64 * q] : make_float2(0.f, 0.f);
        yb[q] = in ? yp[4 * q] : make_float2(0.f, 0.f);
      }
    }
  };
  // two batches per trip, alternating buffers, so that no registers are
  // copied between batches
  load_batch(0, h0, y0);
  for (int r0 = 0; r0 < B; r0 += 8 * kQ) {
    if (r0 + 4 * kQ < B) load_batch(r0 + 4 * kQ, h1, y1);
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      __builtin_amdgcn_s_setprio(1);
      gram_rowquad(h0[q], y0[q], reG, pG, k1, k2, k3, ysq);
      __builtin_amdgcn_s_setprio(0);
    }
    if (r0 + 4 * kQ >= B) break;
    if (r0 + 8 * kQ < B) load_batch(r0 + 8 * kQ, h0, y0);
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      __builtin_amdgcn_s_setprio(1);
      gram_rowquad(h1[q], y1[q], reG, pG, k1, k2, k3, ysq);
      __builtin_amdgcn_s_setprio(0);
    }
  }
  prep_finish(a, grp, active, reG, pG, k1 + k3, k1 + k2, ysq);
}


// Algorithm 1 for one channel group (one wave), from the state the prep
// kernel left in the workspace.  P selects the arithmetic of the L~ T~
// products: float32 MFMAs (16x16x4, K-steps of four columns skipped where L~
// is zero), or BF16 / FP16 operands with float32 accumulation (16x16x16, one
// MFMA per 16-column tile).  V, the norms, rsqrt and the master copy of L~
// are float32 in every case.
template <int P>
__global__ __launch_bounds__(64) void solve_group_qpsk16(FusedArgs a) {
  const int lane = threadIdx.x;
  const int n = lane & 15;
  const int g = lane >> 4;
  const long long v = (long long)blockIdx.x * 16 + n;
  const float* ws = a.ws + (long long)blockIdx.x * kWsFloats;
  constexpr bool k16 = P != TASER_PREC_F32;
  float A[2][2][4], ct[2][4], Dc[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const float re = ws[kWsR + s * 64 + lane], im = ws[kWsM + s * 64 + lane];
    A[0][0][s] = re;
    A[0][1][s] = -im;
    A[1][0][s] = im;
    A[1][1][s] = re;
  }
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) ct[mt][r] = ws[kWsC + (mt * 4 + r) * 64 + lane];
#pragma unroll
  for (int r = 0; r < 4; ++r) Dc[r] = ws[kWsD + 4 * r + g];
  const float DN = ws[kWsDN + n];
  const float tau = ws[kWsTau + n];
  const int fl = __float_as_int(ws[kWsFlag + n]);
  const bool nonfinite = (fl & 2) != 0;
  const bool skip = fl != 0;
  const float m2tau = -2.f * tau;
  // The register of row i that holds the diagonal (columns 4 (i / 4) + g)
  // has lanes above the diagonal, g > i % 4.  There L~ is zero, so a zero
  // step factor keeps V zero without a select: mdiag[d] is the factor for
  // rows with i % 4 == d.
  float mdiag[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) mdiag[d] = g <= d ? m2tau : 0.f;
  // float32 path: [V0; V1] = [R -M; M R] [a; b] is the complex product
  // (R + jM)(a + jb), formed with three real products (Gauss):
  // P1 = R a, P2 = M b, P3 = (R + M)(a + b); V0 = P1 - P2, V1 = P3 - P1 - P2.
  float Apm[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) Apm[s] = A[0][0][s] + A[1][0][s];
  u2 Ah[2][2];
  if constexpr (k16) {
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int kt = 0; kt < 2; ++kt)
        Ah[mt][kt] = pack4<P>(A[mt][kt][0], A[mt][kt][1], A[mt][kt][2], A[mt][kt][3]);
  }

  // ---------------- Algorithm 1: L~(0) = D, t_max FBS steps ----------------
  // Lr[i][mt][r] is stored only where 16 mt + 4 r <= i (otherwise the whole
  // register is in the strictly upper triangle for every lane).
  float Lr[32][2][4];
  float l21[2][4];
  float l22 = DN;
  sfor<0, 32>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    sfor<0, 2>([&](auto mc) {
      constexpr int MT = decltype(mc)::value;
      sfor<0, 4>([&](auto rc) {
        constexpr int R = decltype(rc)::value;
        if constexpr (16 * MT + 4 * R <= I) {
          const int j = 16 * MT + 4 * R + g;
          Lr[I][MT][R] = (j == I) ? Dc[R] : 0.f;
        }
      });
    });
  });
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) l21[mt][r] = 0.f;

  const bool pin = !(a.flags & TASER_FLAG_LITERAL_LAST);
  int st_bits = 0;
  const int iters = a.t_max;
  for (int t = 0; t < iters; ++t) {
    float nsq[2][4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) nsq[mt][r] = 0.f;

    // Products of every row are independent (row i of V needs row i of L~
    // only), so the MFMAs run ahead of the VALU epilogue: the last row's
    // product is issued first and each row's epilogue trails the products
    // of the next kAhead rows.
    constexpr int kAhead = 2;
    f4 lacc[2];
    if constexpr (k16) {
      const u2 b0 = pack4<P>(l21[0][0], l21[0][1], l21[0][2], l21[0][3]);
      const u2 b1 = pack4<P>(l21[1][0], l21[1][1], l21[1][2], l21[1][3]);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        lacc[mt] = mfma32<P>(Ah[mt][0], Ah[mt][1], b0, b1, f4{0.f, 0.f, 0.f, 0.f});
      }
    } else {
      f4 p1 = {0.f, 0.f, 0.f, 0.f}, p2 = p1, p3 = p1;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        p1 = mfma(A[0][0][s], l21[0][s], p1);
        p2 = mfma(A[1][0][s], l21[1][s], p2);
        p3 = mfma(Apm[s], l21[0][s] + l21[1][s], p3);
      }
      lacc[0] = p1 - p2;
      lacc[1] = p3 - p1 - p2;
    }
    float cl = 0.f;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) cl += l21[mt][r] * ct[mt][r];

    f4 ring[kAhead + 1][2];
    auto product = [&](auto ic) {
      constexpr int I = decltype(ic)::value;
      constexpr int SLOT = I % (kAhead + 1);
      if constexpr (k16) {
        auto Lv = [&](auto kc, auto rc) {
          constexpr int KT = decltype(kc)::value, R = decltype(rc)::value;
          if constexpr (16 * KT + 4 * R <= I) return Lr[I][KT][R];
          else return 0.f;
        };
        using C0 = std::integral_constant<int, 0>;
        using C1 = std::integral_constant<int, 1>;
        using C2 = std::integral_constant<int, 2>;
        using C3 = std::integral_constant<int, 3>;
        const u2 b0 = pack4<P>(Lv(C0{}, C0{}), Lv(C0{}, C1{}), Lv(C0{}, C2{}), Lv(C0{}, C3{}));
        if constexpr (I >= 16) {
          // both column tiles of the row are nonzero: one K = 32 product per
          // output tile
          const u2 b1 = pack4<P>(Lv(C1{}, C0{}), Lv(C1{}, C1{}), Lv(C1{}, C2{}), Lv(C1{}, C3{}));
          ring[SLOT][0] = mfma32<P>(Ah[0][0], Ah[0][1], b0, b1, f4{0.f, 0.f, 0.f, 0.f});
          ring[SLOT][1] = mfma32<P>(Ah[1][0], Ah[1][1], b0, b1, f4{0.f, 0.f, 0.f, 0.f});
        } else {
          ring[SLOT][0] = mfma16<P>(Ah[0][0], b0, f4{0.f, 0.f, 0.f, 0.f});
        }
        return;
      }
      if constexpr (I < 16) {
        // one column tile: V0 = R a over the K-steps at or below the diagonal
        ring[SLOT][0] = f4{0.f, 0.f, 0.f, 0.f};
        sfor<0, 4>([&](auto sc) {
          constexpr int S = decltype(sc)::value;
          if constexpr (4 * S <= I) ring[SLOT][0] = mfma(A[0][0][S], Lr[I][0][S], ring[SLOT][0]);
        });
      } else {
        // a = tile 0 (full), b = tile 1 (K-steps up to the diagonal)
        f4 p1 = {0.f, 0.f, 0.f, 0.f}, p2 = p1, p3 = p1;
        sfor<0, 4>([&](auto sc) {
          constexpr int S = decltype(sc)::value;
          p1 = mfma(A[0][0][S], Lr[I][0][S], p1);
          if constexpr (16 + 4 * S <= I) {
            p2 = mfma(A[1][0][S], Lr[I][1][S], p2);
            p3 = mfma(Apm[S], Lr[I][0][S] + Lr[I][1][S], p3);
          } else {
            p3 = mfma(Apm[S], Lr[I][0][S], p3);
          }
        });
        ring[SLOT][0] = p1 - p2;
        ring[SLOT][1] = p3 - p1 - p2;
      }
    };
    auto epilogue = [&](auto ic) {
      constexpr int I = decltype(ic)::value;
      constexpr int SLOT = I % (kAhead + 1);
      sfor<0, 2>([&](auto mc) {
        constexpr int MT = decltype(mc)::value;
        sfor<0, 4>([&](auto rc) {
          constexpr int R = decltype(rc)::value;
          if constexpr (16 * MT + 4 * R <= I) {
            float m = m2tau;
            if constexpr (16 * MT + 4 * R + 3 > I) m = mdiag[I - 16 * MT - 4 * R];
            const float x = fmaf(m, ring[SLOT][MT][R], Lr[I][MT][R]);
            Lr[I][MT][R] = x;
            nsq[MT][R] = fmaf(x, x, nsq[MT][R]);
          }
        });
      });
    };
    sfor<0, kAhead>([&](auto ic) { product(ic); });
    sfor<0, 32>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      // the wave issuing its next row's MFMAs gets issue priority over a
      // wave in its vector-ALU epilogue, which keeps the matrix pipe fed
      if constexpr (I + kAhead < 32) {
        __builtin_amdgcn_s_setprio(1);
        product(std::integral_constant<int, I + kAhead>{});
        __builtin_amdgcn_s_setprio(0);
      }
      epilogue(ic);
    });

    // last row: V = l21 - 2 tau (l21^T G~ + l22 c~^T), and V_NN
    cl = sum_groups(cl);
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float x = fmaf(m2tau, fmaf(l22, ct[mt][r], lacc[mt][r]), l21[mt][r]);
        l21[mt][r] = x;
        nsq[mt][r] = fmaf(x, x, nsq[mt][r]);
      }
    const float vnn = fmaf(m2tau, cl + l22, l22);   // T~_NN = 1
    if (!(vnn > 0.f)) st_bits |= TASER_VEC_VNN_NONPOS;

    // prox: column j <- D_j V_:,j / ||V_:,j||
    float sc[2][4];
    bool any_bad = false;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float q = nsq[mt][r];
        const bool ok = q > 0.f && q < 3.4e38f;
        sc[mt][r] = ok ? Dc[r] * __builtin_amdgcn_rsqf(q) : 0.f;
        any_bad |= !ok;
      }
    sfor<0, 32>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      sfor<0, 2>([&](auto mc) {
        constexpr int MT = decltype(mc)::value;
        sfor<0, 4>([&](auto rc) {
          constexpr int R = decltype(rc)::value;
          if constexpr (16 * MT + 4 * R <= I) Lr[I][MT][R] *= sc[MT][R];
        });
      });
    });
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) l21[mt][r] *= sc[mt][r];
    if (__builtin_expect(__ballot(any_bad) != 0ull, 0)) {
      // reset columns with zero / non-finite norm to D_jj e_j
      if (any_bad) st_bits |= TASER_VEC_ZERO_NORM;
      sfor<0, 32>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        constexpr int MT = I / 16, R = (I % 16) / 4;
        if (sc[MT][R] == 0.f && g == (I & 3)) Lr[I][MT][R] = Dc[R];
      });
    }
    if (pin) {
      l22 = DN;
    } else if (vnn != 0.f && isfinite(vnn)) {
      l22 = vnn > 0.f ? DN : -DN;
    } else {
      l22 = DN;
      st_bits |= TASER_VEC_ZERO_NORM;
    }
  }

  // ---------------- slicing and outputs ----------------
  int bits = or_groups(st_bits);
  if (skip) bits = nonfinite ? TASER_VEC_NONFINITE : TASER_VEC_DEGENERATE;

  int8_t* sb = a.sbar + v * 32;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = 16 * mt + 4 * r + g;
      const float x = skip ? 0.f : l21[mt][r];
      sb[j] = x >= 0.f ? (int8_t)1 : (int8_t)-1;
      if (a.margin) a.margin[v * 32 + j] = skip ? 0.f : x / Dc[r];
    }
  if (g == 0) a.status[v] = bits;
  if (a.L_out) {
    float* Lo = a.L_out + v * 561;
    sfor<0, 32>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      sfor<0, 2>([&](auto mc) {
        constexpr int MT = decltype(mc)::value;
        sfor<0, 4>([&](auto rc) {
          constexpr int R = decltype(rc)::value;
          if constexpr (16 * MT + 4 * R <= I) {
            const int j = 16 * MT + 4 * R + g;
            if (j <= I) {
              float x = Lr[I][MT][R];
              if (skip) x = (j == I) ? (nonfinite ? 1.f : Dc[R]) : 0.f;
              Lo[I * (I + 1) / 2 + j] = x;
            }
          }
        });
      });
    });
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) Lo[528 + 16 * mt + 4 * r + g] = skip ? 0.f : l21[mt][r];
    if (g == 0) Lo[560] = skip ? (nonfinite ? 1.f : DN) : l22;
  }
}

}  // namespace

bool fused_group_supported(const FusedArgs& a) {
  return a.mode == TASER_COHERENT && a.mod == TASER_QPSK && a.U == 16 && a.y_per_H % 16 == 0 &&
         a.B >= 1;
}

bool fused_supported(const FusedArgs& a) {
  return fused_group_supported(a) || fused_vec_tiles(a) > 0;
}

size_t fused_workspace_bytes(const FusedArgs& a) {
  return fused_group_supported(a) ? (size_t)(a.V / 16) * kWsFloats * sizeof(float) : 0;
}

hipError_t launch_fused_prep(const FusedArgs& a, hipStream_t s) {
  const int groups = a.V / 16;
  hipLaunchKernelGGL(prep_group_qpsk16, dim3((groups + kPrepWaves - 1) / kPrepWaves),
                     dim3(64 * kPrepWaves), 0, s, a, groups);
  return hipGetLastError();
}

hipError_t launch_fused_solve(const FusedArgs& a, hipStream_t s) {
  const int groups = a.V / 16;
  if (a.prec == TASER_PREC_BF16)
    hipLaunchKernelGGL(solve_group_qpsk16<TASER_PREC_BF16>, dim3(groups), dim3(64), 0, s, a);
  else if (a.prec == TASER_PREC_F16)
    hipLaunchKernelGGL(solve_group_qpsk16<TASER_PREC_F16>, dim3(groups), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(solve_group_qpsk16<TASER_PREC_F32>, dim3(groups), dim3(64), 0, s, a);
  return hipGetLastError();
}

// tau[v] of every vector from a prepared workspace (lane n of a group's tau
// row holds vector n).
__global__ __launch_bounds__(256) void read_tau(const float* __restrict__ ws, int V,
                                                float* __restrict__ tau) {
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v < V) tau[v] = ws[(long long)(v / 16) * kWsFloats + kWsTau + (v & 15)];
}

hipError_t launch_fused_tau(const FusedArgs& a, float* tau, hipStream_t s) {
  hipLaunchKernelGGL(read_tau, dim3((a.V + 255) / 256), dim3(256), 0, s, a.ws, a.V, tau);
  return hipGetLastError();
}

hipError_t launch_fused(const FusedArgs& a, hipStream_t s) {
  if (!fused_group_supported(a)) return launch_fused_vec(a, s);
  hipError_t e = launch_fused_prep(a, s);
  if (e != hipSuccess) return e;
  return launch_fused_solve(a, s);
}

}  // namespace taser
