// Fused single-launch TASER for vectors that each have their own T~:
// coherent detection with one channel per vector (or per few vectors) and
// joint channel estimation and detection (Section II-B), BPSK or QPSK, for
// N - 1 <= 16 NT with NT in {1, 2, 4} (padded problems keep their padded
// rows and columns at zero).
//
// One wave detects one vector.  T~ is bordered, T~ = [G~ c~; c~^T t], with
// G~ the (N-1)x(N-1) block.  The L~ T~ product of Algorithm 1 runs on
// 16x16x4 MFMAs with G~ as the A operand (held in NT*NT*4 VGPRs) and a
// 16-row tile of L~ as the B operand: lane l serves row (l % 16) of a row
// tile and column quad g = l / 16, holding columns 16 jt + 4 r + g in
// register (jt, r); the output rows are permuted by jj(m) = 4 (m % 4) + m/4
// so that the product lands in the same layout.  Column norms are sums over
// the 16 rows of each tile (DPP within a 16-lane row).  The last row of L~
// and the Lanczos vectors of the step-size estimate are handled as
// matrix-vector products through the same A registers on the vector ALUs.
#include <math.h>

#include <mutex>
#include <type_traits>

#include "spectral.h"
#include "taser_internal.h"

namespace taser {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned u2 __attribute__((ext_vector_type(2)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));

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

// One 16x16x32 product: the K slots of two 16-column tiles side by side,
// a = [a0, a1], b = [b0, b1] (the same K order in both operands).  On gfx950
// it takes the cycles of one 16x16x16 product for twice the work.
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

// Sum over the four column quads (lanes n, n+16, n+32, n+48).
__device__ __forceinline__ float sum_quads(float x) {
  const unsigned u = __float_as_uint(x);
  const auto h = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  const float y = __uint_as_float(h[0]) + __uint_as_float(h[1]);
  const unsigned w = __float_as_uint(y);
  const auto r = __builtin_amdgcn_permlane16_swap(w, w, false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Sum over the 16 lanes of each 16-lane row (the rows of a tile), by
// rotations inside the row (DPP row_ror).
__device__ __forceinline__ float sum_rows16(float x) {
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xF, 0xF, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x124, 0xF, 0xF, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x122, 0xF, 0xF, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x121, 0xF, 0xF, false));
  return x;
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  // every lane of a row has a valid source for the controls used here, so
  // bound_ctrl (0 for an invalid source) never applies; it spares the
  // compiler a zero-initialised destination register per move
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}

// Sum over the N1 = 16, 32 or 64 entries of a vector held one entry per lane
// (lane l holds entry l mod N1), with the same bits in every lane: each level
// pairs two lanes that add the same two partial sums (lane ^ 1, lane ^ 2,
// the half-row and row mirrors, then the gfx950 row swaps).  A rotation
// tree would give every lane its own order of additions, and the copies of
// the Lanczos vector would drift apart.
template <int N1>
__device__ __forceinline__ float sum_lanes(float x) {
  // x rounded in its register first: a product contracted into the first
  // addition would be exact in one lane of a pair and rounded in the other
  asm volatile("" : "+v"(x));
  x += dpp_f<0xB1>(x);    // quad_perm [1, 0, 3, 2]
  x += dpp_f<0x4E>(x);    // quad_perm [2, 3, 0, 1]
  x += dpp_f<0x141>(x);   // row_half_mirror
  x += dpp_f<0x140>(x);   // row_mirror
  if constexpr (N1 >= 64) {
    const unsigned u = __float_as_uint(x);
    const auto h = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    x = __uint_as_float(h[0]) + __uint_as_float(h[1]);
  }
  if constexpr (N1 >= 32) {
    const unsigned u = __float_as_uint(x);
    const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    x = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  return x;
}

// One level of a transpose-reduction inside 16-lane rows: each lane swaps
// half of its K values with its DPP partner (an involution of the row) and
// keeps the half that `upper` selects, summed with the partner's copy.
template <int K, int CTRL>
__device__ __forceinline__ void halve_rows16(float* x, bool upper) {
#pragma unroll
  for (int a = 0; a < K / 2; ++a) {
    const float keep = upper ? x[a + K / 2] : x[a];
    const float send = upper ? x[a] : x[a + K / 2];
    x[a] = keep + dpp_f<CTRL>(send);
  }
}

// Sums of M values over the 16 lanes of each row, lane n of a row ending
// with the sum for value c = n / (16 / M).  Partners, in order: n ^ 8
// (row_ror:8), 7 - n within each half-row (row_half_mirror), n ^ 2 and
// n ^ 1 (quad permutations); each pairs lanes whose partial sums cover
// disjoint lane sets.  The levels that halve use the lane bits that make up
// c; once one value is left the remaining partners add whole values.  About
// 3 M / 2 instructions instead of the 4 M of a row all-reduce per value.
template <int M>
__device__ __forceinline__ float reduce_rows16(float (&x)[M], int n) {
  constexpr int kRor8 = 0x128, kHalfMirror = 0x141, kXor2 = 0x4E, kXor1 = 0xB1;
  if constexpr (M >= 2) halve_rows16<M, kRor8>(x, (n & 8) != 0);
  if constexpr (M >= 4) halve_rows16<M / 2, kHalfMirror>(x, (n & 4) != 0);
  if constexpr (M >= 8) halve_rows16<M / 4, kXor2>(x, (n & 2) != 0);
  if constexpr (M >= 16) halve_rows16<M / 8, kXor1>(x, (n & 1) != 0);
  float s = x[0];
  if constexpr (M < 16) s += dpp_f<kXor1>(s);
  if constexpr (M < 8) s += dpp_f<kXor2>(s);
  if constexpr (M < 4) s += dpp_f<kHalfMirror>(s);
  if constexpr (M < 2) s += dpp_f<kRor8>(s);
  return s;
}

// Lane LANE's value broadcast to every lane of its 16-lane row
// (row_newbcast).
template <int LANE>
__device__ __forceinline__ float row_bcast(float x) {
  return dpp_f<0x150 + LANE>(x);
}

__device__ __forceinline__ int or_all(int x) {
  return __ballot(x != 0) != 0ull;
}

// Hardware reciprocal, square root and reciprocal square root (about one
// ulp; the correctly rounded library forms cost some twenty instructions).
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float hsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Largest eigenvalue of the symmetric tridiagonal (al, b2 = beta^2), the same
// in every lane, by 65-way multisection: in each round lane l tests the
// point lo + (l + 1)(hi - lo)/65 with a Sturm count (the number of
// eigenvalues below it).  Plain float32 Lanczos repeats converged Ritz values
// (loss of orthogonality), and counting is insensitive to such clusters.
// The bracket is [max_k al_k, Gershgorin upper bound]: diagonal entries are
// Rayleigh quotients, so the largest one bounds the top eigenvalue below.
template <int M>
__device__ __forceinline__ float top_eigenvalue(const float* al, const float* b2) {
  float lo = -3.4e38f, hi = -3.4e38f;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const float rad = (k > 0 ? hsqrt(b2[k - 1]) : 0.f) + (k < M - 1 ? hsqrt(b2[k]) : 0.f);
    hi = fmaxf(hi, al[k] + rad);
    lo = fmaxf(lo, al[k]);
  }
  const float pivmin = 1e-30f + 1e-12f * fabsf(hi);
  const int lane = threadIdx.x & 63;
  for (int round = 0; round < 5; ++round) {
    const float w = (hi - lo) * (1.f / 65.f);
    const float x = lo + w * (float)(lane + 1);
    int cnt = 0;
    float d = al[0] - x;
    if (fabsf(d) < pivmin) d = -pivmin;
    cnt += d < 0.f;
#pragma unroll
    for (int k = 1; k < M; ++k) {
      d = (al[k] - x) - b2[k - 1] * rcp(d);
      if (fabsf(d) < pivmin) d = -pivmin;
      cnt += d < 0.f;
    }
    const unsigned long long hit = __ballot(cnt >= M);   // every eigenvalue below x
    const int first = hit ? __ffsll((long long)hit) - 1 : 64;
    const float nlo = lo + w * (float)first;
    hi = first < 64 ? lo + w * (float)(first + 1) : hi;
    lo = nlo;
    // a bracket within 1e-7 of the value is below what float32 Lanczos
    // resolves (about 1e-6); most brackets get there in three or four rounds
    if (!(hi - lo > 1e-7f * fabsf(hi))) break;
  }
  return 0.5f * (lo + hi);
}

// The same, for a tridiagonal held one entry per lane (lane k: al_k, b2_k;
// lanes past the last step hold -1e30 and 0, which count like a breakdown):
// the M leading entries are read into scalars.
template <int M>
__device__ __forceinline__ float top_eigenvalue_lanes(float alv, float b2v) {
  float al[M], b2[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    al[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(alv), k));
    b2[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(b2v), k));
  }
  return top_eigenvalue<M>(al, b2);
}

// Most Lanczos steps a problem of NT tiles takes (the kernels serve U <= 32,
// so real problems stop at N = 33), and the top eigenvalue of m <= that
// many entries.
template <int NT>
constexpr int kVecLanczosCap =
    spectral::lanczos_steps(16 * NT + 1 < 33 ? 16 * NT + 1 : 33, false) >
            spectral::lanczos_steps(16 * NT + 1, true)
        ? spectral::lanczos_steps(16 * NT + 1 < 33 ? 16 * NT + 1 : 33, false)
        : spectral::lanczos_steps(16 * NT + 1, true);

template <int NT>
__device__ __forceinline__ float ritz_top(float alv, float b2v, int m) {
  static_assert(kVecLanczosCap<NT> <= 24, "Ritz entries beyond the multisections");
  if (m <= 8) return top_eigenvalue_lanes<8>(alv, b2v);
  if (m <= 16) return top_eigenvalue_lanes<16>(alv, b2v);
  return top_eigenvalue_lanes<24>(alv, b2v);
}

// A value that is the same in every lane, as a scalar.
__device__ __forceinline__ float uniform(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// The padded T is symmetric: its lower triangle is kept packed by rows
// (half the LDS of the square, which doubles the waves a CU holds for the
// four-tile kernels).
template <int NT>
struct VecLds {
  static constexpr int N1 = 16 * NT;
  static constexpr int TT = (N1 + 1) * (N1 + 2) / 2;             // packed padded T
  static constexpr int REGION = TT;
  static constexpr int FLOATS = REGION + (N1 + 1) + N1;          // + D + shuffle buffer
};

// Entry (i, j) of the packed symmetric T, either order.
__device__ __forceinline__ int tix(int i, int j) {
  const int hi = i > j ? i : j, lo = i > j ? j : i;
  return hi * (hi + 1) / 2 + lo;
}

// One vector's problem: where its inputs and outputs are and its sizes.
struct VecJob {
  long long v;            // vector index (status, tau_in)
  int B, U, N, mod;
  const float2* H;        // coherent: B x U row-major channel; JED: unused
  const float2* y;        // coherent: y (B); JED: Y (U+1 slots x B)
  float2 s0;              // JED pilot
  int8_t* sbar;           // N-1 decisions
  float* margin;          // N-1 margins or NULL
  float* L;               // packed L~ or NULL
  int pad_to;             // mixed batches: entries N-1 .. pad_to-1 of sbar/margin are set to 0
};

// T (eq. (2) coherent, eq. (5) joint detection) of one vector into LDS T
// [(16 NT + 1)^2] in padded indexing (real index i < N - 1 -> i, N - 1 ->
// 16 NT; the padding rows and columns are zero).  One wave; ends with a
// barrier.
template <int NT, int P, bool GAUSS>
__device__ __forceinline__ void vec_build_T(const VecJob& job, bool jed, float* T) {
  constexpr int N1 = 16 * NT;
  using S = VecLds<NT>;
  const int lane = threadIdx.x;
  const int n = lane & 15;
  const int g = lane >> 4;
  const int B = job.B, U = job.U;
  const bool qpsk = job.mod == TASER_QPSK;
  const float sg = jed ? -1.f : 1.f;

  // ---------------- preprocessing: complex Gram, H^H y, ||y||^2 ----------------
  // G = H^H H on 16x16x4 MFMAs, streamed from HBM: for row-quad q, lane
  // (n, g) holds h_t = H[4 q + g][16 t + n] (user tile t); Re G and Im G of
  // user tiles (t1, t2) accumulate from h_t1 (A) and h_t2 (B), only t1 >= t2
  // (G is Hermitian).  H^H y and ||y||^2 are lane partial sums over the
  // lane's rows, reduced over the four row lanes afterwards.  For joint
  // detection H is Y_r = [y_1 .. y_K] and y is y_0 s_0.
  constexpr int UTM = NT >= 2 ? 2 : 1;         // user tiles (U <= 16 NT, U <= 32)
  const int UT = U > 16 ? 2 : 1;
  const float2* Hg = job.H;
  const float2* yg = job.y;
  const float2 s0 = job.s0;
  auto hval = [&](int row, int u) {
    if (row >= B || u >= U) return make_float2(0.f, 0.f);
    return jed ? yg[(long long)(u + 1) * B + row] : Hg[(long long)row * U + u];
  };
  auto yval = [&](int row) {
    if (row >= B) return make_float2(0.f, 0.f);
    const float2 y0 = yg[row];
    if (!jed) return y0;
    return make_float2(y0.x * s0.x - y0.y * s0.y, y0.x * s0.y + y0.y * s0.x);
  };
  // tiles (0,0), (1,0), (1,1).  QPSK with GAUSS: Gauss's three real products
  // per complex tile; for conj(a + jb) (c + jd), k1 = (a - b) c,
  // k2 = a (d - c), k3 = b (c + d), so Re = k1 + k3 and Im = ad - bc = k1 + k2
  // (gre holds k1, gim k2, gk3 k3).  It saves a quarter of the Gram MFMAs but
  // needs a third set of accumulators: the four-tile kernels use it (every
  // variant of a size takes the same arithmetic, so launch choices do not
  // change results); with one or two tiles the spills of the five-wave
  // budget cost more than the products saved, and the four products of Re
  // and Im are taken directly.  BPSK needs only Re G (two products into gre).
  f4 gre[3], gim[3], gk3[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) { gre[k] = f4{0.f, 0.f, 0.f, 0.f}; gim[k] = gre[k]; gk3[k] = gre[k]; }
  float bre[UTM], bim[UTM], ysq = 0.f;
#pragma unroll
  for (int t = 0; t < UTM; ++t) { bre[t] = 0.f; bim[t] = 0.f; }
  // row-quads per batch (double-buffered): the four-tile kernels have
  // registers to spare in this phase (their peak is the loop's L~ tiles), and
  // a deeper prefetch covers more of the load latency of a 64 KB channel
  constexpr int kQ = NT == 4 ? 8 : 4;
  float2 hc[kQ][UTM], yc[kQ], hn[kQ][UTM], yn[kQ];
  auto load_batch = [&](int q0, float2 (&hb)[kQ][UTM], float2 (&yb)[kQ]) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int row = 4 * (q0 + q) + g;
#pragma unroll
      for (int t = 0; t < UTM; ++t) hb[q][t] = t < UT ? hval(row, 16 * t + n) : make_float2(0.f, 0.f);
      yb[q] = yval(row);
    }
  };
  const int quads = (B + 3) / 4;
  // BPSK needs only Re G and Re b (T uses the real parts), so its row loop
  // issues half the Gram MFMAs; the modulation is the same in every lane
  auto rows = [&](auto qc) {
    constexpr bool Q = decltype(qc)::value;
    load_batch(0, hc, yc);
    for (int q0 = 0; q0 < quads; q0 += kQ) {
      if (q0 + kQ < quads) load_batch(q0 + kQ, hn, yn);
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const float2 h0 = hc[q][0], y = yc[q];
        // float32 products: issue priority while this wave feeds the matrix
        // pipe (here and in the tril products below); with 16-bit products it
        // made mixed batches slower
        if constexpr (P == TASER_PREC_F32) __builtin_amdgcn_s_setprio(1);
        if constexpr (Q && GAUSS) {
          // A side (a - b), a, b of the left tile; B side c, (d - c), (c + d)
          // of the right tile
          const float amb0 = h0.x - h0.y, dmc0 = h0.y - h0.x, cpd0 = h0.x + h0.y;
          gre[0] = mfma(amb0, h0.x, gre[0]);
          gim[0] = mfma(h0.x, dmc0, gim[0]);
          gk3[0] = mfma(h0.y, cpd0, gk3[0]);
          if constexpr (UTM == 2) {
            if (UT == 2) {
              const float2 h1 = hc[q][1];
              const float amb1 = h1.x - h1.y, dmc1 = h1.y - h1.x, cpd1 = h1.x + h1.y;
              gre[1] = mfma(amb1, h0.x, gre[1]);
              gim[1] = mfma(h1.x, dmc0, gim[1]);
              gk3[1] = mfma(h1.y, cpd0, gk3[1]);
              gre[2] = mfma(amb1, h1.x, gre[2]);
              gim[2] = mfma(h1.x, dmc1, gim[2]);
              gk3[2] = mfma(h1.y, cpd1, gk3[2]);
            }
          }
        } else {
          gre[0] = mfma(h0.x, h0.x, gre[0]);     // Re G = Hr^T Hr + Hi^T Hi
          gre[0] = mfma(h0.y, h0.y, gre[0]);
          if constexpr (Q) {
            gim[0] = mfma(h0.x, h0.y, gim[0]);   // Im G = Hr^T Hi - Hi^T Hr
            gim[0] = mfma(h0.y, -h0.x, gim[0]);
          }
          if constexpr (UTM == 2) {
            if (UT == 2) {
              const float2 h1 = hc[q][1];
              gre[1] = mfma(h1.x, h0.x, gre[1]);
              gre[1] = mfma(h1.y, h0.y, gre[1]);
              gre[2] = mfma(h1.x, h1.x, gre[2]);
              gre[2] = mfma(h1.y, h1.y, gre[2]);
              if constexpr (Q) {
                gim[1] = mfma(h1.x, h0.y, gim[1]);
                gim[1] = mfma(h1.y, -h0.x, gim[1]);
                gim[2] = mfma(h1.x, h1.y, gim[2]);
                gim[2] = mfma(h1.y, -h1.x, gim[2]);
              }
            }
          }
        }
        if constexpr (P == TASER_PREC_F32) __builtin_amdgcn_s_setprio(0);
#pragma unroll
        for (int t = 0; t < UTM; ++t) {          // conj(h) y
          bre[t] = fmaf(hc[q][t].x, y.x, fmaf(hc[q][t].y, y.y, bre[t]));
          if constexpr (Q) bim[t] = fmaf(hc[q][t].x, y.y, fmaf(-hc[q][t].y, y.x, bim[t]));
        }
        ysq = fmaf(y.x, y.x, fmaf(y.y, y.y, ysq));
      }
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        yc[q] = yn[q];
#pragma unroll
        for (int t = 0; t < UTM; ++t) hc[q][t] = hn[q][t];
      }
    }
  };
  if (qpsk) {
    rows(std::true_type{});
    if constexpr (GAUSS) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const f4 k1 = gre[k];
        gre[k] = k1 + gk3[k];
        gim[k] = k1 + gim[k];
      }
    }
  } else {
    rows(std::false_type{});
  }
#pragma unroll
  for (int t = 0; t < UTM; ++t) { bre[t] = sum_quads(bre[t]); bim[t] = sum_quads(bim[t]); }
  ysq = sum_quads(ysq);                        // rows 4 q + g summed over the four g lanes

  // T in padded indexing (eq. (2) coherent, eq. (5) joint detection),
  // lower triangle packed: the lane of entry (p, q) with p >= q writes it
  // (on the diagonal tiles the lane of (q, p) holds the same sums)
  for (int e = lane; e < S::TT; e += 64) T[e] = 0.f;
  __syncthreads();
  auto put_tile = [&](const f4& re4, const f4& im4, int t1, int t2) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int p = 16 * t1 + 4 * g + r, q = 16 * t2 + n;
      if (p >= U || q >= U || p < q) continue;
      const float gr = sg * re4[r], gi = p == q ? 0.f : sg * im4[r];
      T[tix(p, q)] = gr;
      if (qpsk) {
        T[tix(U + p, U + q)] = gr;
        T[tix(U + q, p)] = -gi;                  // T(p, U + q) = -Im G(p, q)
        T[tix(U + p, q)] = gi;
      }
    }
  };
  put_tile(gre[0], gim[0], 0, 0);
  if (UT == 2) {
    put_tile(gre[1], gim[1], 1, 0);
    put_tile(gre[2], gim[2], 1, 1);
  }
  if (g == 0) {
#pragma unroll
    for (int t = 0; t < UTM; ++t) {
      const int p = 16 * t + n;
      if (p < U) {
        // last column: -Hbar^T ybar in both modes
        T[tix(N1, p)] = -bre[t];
        if (qpsk) T[tix(N1, U + p)] = -bim[t];
      }
    }
  }
  if (lane == 0) T[tix(N1, N1)] = sg * ysq;
  __syncthreads();
}

template <int NT, int P, bool GAUSS = (NT == 4)>
__device__ __forceinline__ void vec_body(const FusedArgs& a, const VecJob& job, float* lds) {
  constexpr int N1 = 16 * NT;
  using S = VecLds<NT>;
  float* T = lds;                        // packed, padded index: real i < N-1 -> i, N-1 -> N1
  float* Dl = lds + S::REGION;           // [N1+1]
  float* sh = Dl + (N1 + 1);             // [N1] layout shuffle

  const int lane = threadIdx.x;
  const int n = lane & 15;
  const int g = lane >> 4;
  const long long v = job.v;
  const int B = job.B, U = job.U, Nm1 = job.N - 1;
  const bool jed = a.mode == TASER_JED;
  const bool qpsk = job.mod == TASER_QPSK;
  const float sg = jed ? -1.f : 1.f;

  vec_build_T<NT, P, GAUSS>(job, jed, T);

  // ---------------- Jacobi preconditioning (Section III-C) ----------------
  int bad = 0, deg = 0;
  for (int e = lane; e < S::TT; e += 64)
    if (!isfinite(T[e])) bad = 1;
  const bool nonfinite = or_all(bad);
  for (int k = lane; k <= N1; k += 64) {
    const bool real_k = k < Nm1 || k == N1;
    const float d = nonfinite ? 0.f : fabsf(T[tix(k, k)]);
    if (real_k && d == 0.f) deg = 1;
    Dl[k] = (d == 0.f || !real_k) ? 1.f : hsqrt(d);
  }
  const bool degenerate = !nonfinite && or_all(deg);
  const bool skip = nonfinite || degenerate;
  __syncthreads();
  const float DN = Dl[N1];
  const float iDN = rcp(DN);
  const float tNN = skip ? 0.f : T[tix(N1, N1)] * (iDN * iDN);
  float A[NT][NT][4];
  {
    const int jr = 4 * (n & 3) + (n >> 2);
    sfor<0, NT>([&](auto jc) {
      constexpr int JT = decltype(jc)::value;
      const int j = 16 * JT + jr;
      const float idj = rcp(Dl[j]);
      sfor<0, NT>([&](auto kc) {
        constexpr int KT = decltype(kc)::value;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = 16 * KT + 4 * s + g;
          A[JT][KT][s] = skip ? 0.f : T[tix(j, k)] * (idj * rcp(Dl[k]));
        }
      });
    });
  }
  float ct[NT][4], Dc[NT][4];
  bool act[NT][4];
  sfor<0, NT>([&](auto jc) {
    constexpr int JT = decltype(jc)::value;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = 16 * JT + 4 * r + g;
      act[JT][r] = j < Nm1;
      Dc[JT][r] = Dl[j];
      ct[JT][r] = skip ? 0.f : T[tix(N1, j)] * (rcp(Dl[j]) * iDN);
    }
  });
  // the last column of T~ once more, one entry per lane, for the step
  // size's Lanczos vectors: lane (n, g) holds entry 16 (g mod NT) + jr(n),
  // the row that the matrix registers' row sums leave in that lane
  const int jt_own = g & (NT - 1);
  const int e_own = 16 * jt_own + 4 * (n & 3) + (n >> 2);
  const float ctd = skip ? 0.f : T[tix(N1, e_own)] * (rcp(Dl[e_own]) * iDN);
  __syncthreads();   // T is dead from here on; sh may be reused freely

  // w (row layout, index 16 jt + jj(m) in lane (m, p)) = G~ x, with x in
  // column layout; returned in column layout through the LDS shuffle.
  auto gemv = [&](const float (&x)[NT][4], float (&w)[NT][4]) {
    const int jr = 4 * (n & 3) + (n >> 2);
    sfor<0, NT>([&](auto jc) {
      constexpr int JT = decltype(jc)::value;
      // two partial sums halve the dependent FMA chain
      float p0 = 0.f, p1 = 0.f;
      sfor<0, NT>([&](auto kc) {
        constexpr int KT = decltype(kc)::value;
        p0 = fmaf(A[JT][KT][0], x[KT][0], p0);
        p1 = fmaf(A[JT][KT][1], x[KT][1], p1);
        p0 = fmaf(A[JT][KT][2], x[KT][2], p0);
        p1 = fmaf(A[JT][KT][3], x[KT][3], p1);
      });
      // the four lanes of a quad hold the same sum and store it to the same
      // word (no lane mask between the rows)
      sh[16 * JT + jr] = sum_quads(p0 + p1);
    });
    // one wave: its LDS accesses complete in program order; the barrier keeps
    // the compiler from moving them across
    __builtin_amdgcn_wave_barrier();
    sfor<0, NT>([&](auto jc) {
      constexpr int JT = decltype(jc)::value;
#pragma unroll
      for (int r = 0; r < 4; ++r) w[JT][r] = sh[16 * JT + 4 * r + g];
    });
    __builtin_amdgcn_wave_barrier();
  };
  auto dot = [&](const float (&x)[NT][4], const float (&y)[NT][4]) {
    float s0 = 0.f, s1 = 0.f;
    sfor<0, NT>([&](auto jc) {
      constexpr int JT = decltype(jc)::value;
      s0 = fmaf(x[JT][0], y[JT][0], s0);
      s1 = fmaf(x[JT][1], y[JT][1], s1);
      s0 = fmaf(x[JT][2], y[JT][2], s0);
      s1 = fmaf(x[JT][3], y[JT][3], s1);
    });
    return sum_quads(s0 + s1);
  };

  // ---------------- step size tau = alpha / ||T~||_2 ----------------
  float tau;
  if (a.tau_mode == TASER_TAU_GIVEN) {
    tau = a.tau_in[v];
  } else {
    // Lanczos on sg*T~ (positive semidefinite in both modes) from T~ e_N.
    // The Lanczos vectors are held one entry per lane (the last entry, index
    // N1, as a scalar), so updates and inner products take one instruction
    // per lane; the product with G~ reads the vector in the column layout of
    // the A registers from LDS (the T region, dead by now), and each lane
    // keeps the row sum of its own entry.  Lane J keeps alpha_J and beta_J^2
    // of step J.
    float* xs = lds;
    float q = sg * ctd, qp = 0.f, q32 = sg * tNN, qp32 = 0.f, beta = 0.f;
    const float nrm = sum_lanes<N1>(q * q) + q32 * q32;
    const float inv0 = nrm > 0.f ? rsqrtf(nrm) : 0.f;
    q *= inv0;
    q32 *= inv0;
    float alv = -1e30f, b2v = 0.f, scale = 0.f;
    // spectral::lanczos_steps (joint detection's T~ is the same kind of
    // matrix: the preconditioned Gram of the block with the pilot column),
    // and never more than the dimension of the Krylov space of T~ e_N: that
    // vector lies in the range of T~ (rank at most 2B for BPSK, B complex
    // dimensions for QPSK) and, for QPSK, in the invariant subspace of
    // dimension (N + 1) / 2 of the paired real form.  Plain float32 Lanczos
    // does not see that space close (beta stays at 1e-4 to 1e-2 of the scale
    // instead of vanishing), so steps beyond it would only multiply rounding
    // noise.
    const int kdim = qpsk ? min(job.B, (job.N + 1) / 2) : min(2 * job.B, job.N);
    const int steps = min(spectral::lanczos_steps(job.N, qpsk), kdim);
    for (int J = 0; J < steps; ++J) {
      // w = sg (G~ q + c~ q_N): the copies of an entry store the same word;
      // one wave's LDS accesses complete in program order, and the barrier
      // keeps the compiler from moving them across
      xs[e_own] = q;
      __builtin_amdgcn_wave_barrier();
      float xc[NT][4];
      sfor<0, NT>([&](auto kc) {
        constexpr int KT = decltype(kc)::value;
#pragma unroll
        for (int r = 0; r < 4; ++r) xc[KT][r] = xs[16 * KT + 4 * r + g];
      });
      __builtin_amdgcn_wave_barrier();
      float rs = 0.f;                 // row 16 jt_own + jr(n) of G~ q
      sfor<0, NT>([&](auto jc) {
        constexpr int JT = decltype(jc)::value;
        float p0 = 0.f, p1 = 0.f;
        sfor<0, NT>([&](auto kc) {
          constexpr int KT = decltype(kc)::value;
          p0 = fmaf(A[JT][KT][0], xc[KT][0], p0);
          p1 = fmaf(A[JT][KT][1], xc[KT][1], p1);
          p0 = fmaf(A[JT][KT][2], xc[KT][2], p0);
          p1 = fmaf(A[JT][KT][3], xc[KT][3], p1);
        });
        const float row = sum_quads(p0 + p1);
        rs = jt_own == JT ? row : rs;
      });
      float w = sg * (rs + ctd * q32);
      float w32 = sg * (sum_lanes<N1>(ctd * q) + tNN * q32);
      const float alj = uniform(sum_lanes<N1>(w * q) + w32 * q32);
      w = fmaf(-alj, q, fmaf(-beta, qp, w));
      w32 = fmaf(-alj, q32, fmaf(-beta, qp32, w32));
      const float bb = uniform(sum_lanes<N1>(w * w) + w32 * w32);
      scale = fmaxf(scale, fabsf(alj));
      const bool breakdown = !(bb > 1e-12f * scale * scale);
      if (lane == J) { alv = alj; b2v = breakdown ? 0.f : bb; }
      if (breakdown) break;          // the later entries stay parked
      const float ib = rsq(bb);
      beta = bb * ib;                 // sqrt(bb)
      qp = q;
      q = w * ib;
      qp32 = q32;
      q32 = w32 * ib;
    }
    const float lam = ritz_top<NT>(alv, b2v, steps);
    tau = a.alpha / (lam > 0.f ? lam : 1.f);
  }
  const float m2tau = -2.f * tau;

  // ---------------- Algorithm 1 ----------------
  constexpr bool k16 = P != TASER_PREC_F32;
  constexpr int M = 4 * NT;                    // column registers per lane
  u2 Ah[NT][NT];
  if constexpr (k16) {
    sfor<0, NT>([&](auto jc) {
      constexpr int JT = decltype(jc)::value;
      sfor<0, NT>([&](auto kc) {
        constexpr int KT = decltype(kc)::value;
        Ah[JT][KT] = pack4<P>(A[JT][KT][0], A[JT][KT][1], A[JT][KT][2], A[JT][KT][3]);
      });
    });
  }
  // Lt[it][jt][r]: row 16 it + n, column 16 jt + 4 r + g (jt <= it).  With
  // 16-bit products the last row of L~ is row tile NT (held by the lanes
  // n = 0; the other lanes of that tile stay zero), and its product runs on
  // the matrix cores with the other tiles.  With float32 products it is l21
  // (the same in every lane n), multiplied on the vector ALUs: there the
  // extra 16x16x4 products would cost more matrix time than they save.
  constexpr int RT = k16 ? NT + 1 : NT;
  float Lt[RT][NT][4];
  float l21[NT][4];
  float l22 = DN;
  sfor<0, RT>([&](auto ic) {
    constexpr int IT = decltype(ic)::value;
    sfor<0, (IT < NT ? IT + 1 : NT)>([&](auto jc) {
      constexpr int JT = decltype(jc)::value;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        Lt[IT][JT][r] = (IT == JT && n == 4 * r + g && act[JT][r]) ? Dc[JT][r] : 0.f;
    });
  });
  sfor<0, NT>([&](auto jc) {
    constexpr int JT = decltype(jc)::value;
#pragma unroll
    for (int r = 0; r < 4; ++r) l21[JT][r] = 0.f;
  });
  // Step factor -2 tau, and on the diagonal tiles 0 for the lanes above the
  // diagonal (L~ is zero there, so V stays zero without a select).
  float mdg[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) mdg[r] = (4 * r + g > n) ? 0.f : m2tau;
  // c~ where the last row lives (16-bit path: lanes n = 0 only)
  float ce[NT][4];
  sfor<0, NT>([&](auto jc) {
    constexpr int JT = decltype(jc)::value;
#pragma unroll
    for (int r = 0; r < 4; ++r) ce[JT][r] = (k16 && n != 0) ? 0.f : ct[JT][r];
  });
  // After the column-norm reduction lane n holds column c = n / (16 / M) of
  // its 16-lane row: register (c / 4, c % 4), i.e. column 16 (c / 4) +
  // 4 (c % 4) + g.
  const int cown = n / (16 / M);
  const int jown = 16 * (cown / 4) + 4 * (cown % 4) + g;
  const float Down = Dl[jown];
  const bool aown = jown < Nm1;
  const float f0 = n == 0 ? 1.f : 0.f;         // float32 path: the replicated last row counts once
  const bool pin = !(a.flags & TASER_FLAG_LITERAL_LAST);
  int st_bits = 0;
  const int iters = skip ? 0 : a.t_max;
  for (int t = 0; t < iters; ++t) {
    float nsq[NT][4];
    sfor<0, NT>([&](auto jc) {
      constexpr int JT = decltype(jc)::value;
#pragma unroll
      for (int r = 0; r < 4; ++r) nsq[JT][r] = 0.f;
    });
    // last row's product (float32 path) and c~ . l21 (for V_NN), both from
    // the old last row
    float lw[NT][4];
    float cl;
    if constexpr (k16) {
      float part = 0.f;
      sfor<0, NT>([&](auto jc) {
        constexpr int JT = decltype(jc)::value;
#pragma unroll
        for (int r = 0; r < 4; ++r) part = fmaf(Lt[NT][JT][r], ce[JT][r], part);
      });
      // lanes n = 0 hold the last row; lane 0 has the sum over its four
      cl = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(sum_quads(part))));
    } else {
      gemv(l21, lw);
      cl = dot(l21, ct);
    }
    // V = L~ - 2 tau tril(L~ T~), row tile by row tile
    sfor<0, RT>([&](auto ic) {
      constexpr int IT = decltype(ic)::value;
      constexpr int TM = IT < NT ? IT : NT - 1;      // last column / K tile with nonzero entries
      f4 acc[TM + 1];
      if constexpr (P == TASER_PREC_F32) __builtin_amdgcn_s_setprio(1);
      if constexpr (k16) {
        u2 bk[TM + 1];
        sfor<0, TM + 1>([&](auto kc) {
          constexpr int KT = decltype(kc)::value;
          bk[KT] = pack4<P>(Lt[IT][KT][0], Lt[IT][KT][1], Lt[IT][KT][2], Lt[IT][KT][3]);
        });
        // K tiles in pairs on 16x16x32 products (the cycles of one 16x16x16)
        sfor<0, TM + 1>([&](auto jc) {
          constexpr int JT = decltype(jc)::value;
          acc[JT] = f4{0.f, 0.f, 0.f, 0.f};
          sfor<0, (TM + 2) / 2>([&](auto pc) {
            constexpr int K0 = 2 * decltype(pc)::value;
            if constexpr (K0 + 1 <= TM)
              acc[JT] = mfma32<P>(Ah[JT][K0], Ah[JT][K0 + 1], bk[K0], bk[K0 + 1], acc[JT]);
            else
              acc[JT] = mfma16<P>(Ah[JT][K0], bk[K0], acc[JT]);
          });
        });
      } else {
        sfor<0, TM + 1>([&](auto jc) {
          constexpr int JT = decltype(jc)::value;
          acc[JT] = f4{0.f, 0.f, 0.f, 0.f};
          sfor<0, TM + 1>([&](auto kc) {
            constexpr int KT = decltype(kc)::value;
#pragma unroll
            for (int s = 0; s < 4; ++s) acc[JT] = mfma(A[JT][KT][s], Lt[IT][KT][s], acc[JT]);
          });
        });
      }
      if constexpr (P == TASER_PREC_F32) __builtin_amdgcn_s_setprio(0);
      sfor<0, TM + 1>([&](auto jc) {
        constexpr int JT = decltype(jc)::value;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float x;
          if constexpr (IT == NT)         // last row: V = l21 - 2 tau (l21^T G~ + l22 c~^T)
            x = fmaf(m2tau, fmaf(l22, ce[JT][r], acc[JT][r]), Lt[IT][JT][r]);
          else if constexpr (IT == JT)
            x = fmaf(mdg[r], acc[JT][r], Lt[IT][JT][r]);
          else
            x = fmaf(m2tau, acc[JT][r], Lt[IT][JT][r]);
          Lt[IT][JT][r] = x;
          nsq[JT][r] = fmaf(x, x, nsq[JT][r]);
        }
      });
    });
    if constexpr (!k16) {
      sfor<0, NT>([&](auto jc) {
        constexpr int JT = decltype(jc)::value;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float x = fmaf(m2tau, fmaf(l22, ct[JT][r], lw[JT][r]), l21[JT][r]);
          l21[JT][r] = x;
          nsq[JT][r] = fmaf(x * f0, x, nsq[JT][r]);
        }
      });
    }
    const float vnn = fmaf(m2tau, fmaf(l22, tNN, cl), l22);
    if (!(vnn > 0.f)) st_bits |= TASER_VEC_VNN_NONPOS;
    // prox: column j <- D_j V_:,j / ||V_:,j||.  The squared norms are summed
    // over the 16 lanes of each row by a transpose-reduction (each level
    // halves the values a lane keeps), so that every lane ends with the norm
    // of one column; the scale factors go back by row broadcasts.
    float flat[M];
    sfor<0, NT>([&](auto jc) {
      constexpr int JT = decltype(jc)::value;
#pragma unroll
      for (int r = 0; r < 4; ++r) flat[4 * JT + r] = nsq[JT][r];
    });
    const float q = reduce_rows16<M>(flat, n);
    const bool ok = __builtin_amdgcn_classf(q, 0x180);   // positive normal or subnormal
    const float sown = ok ? Down * __builtin_amdgcn_rsqf(q) : 0.f;
    const bool any_bad = __ballot(aown && !ok) != 0ull;
    float sc[NT][4];
    sfor<0, NT>([&](auto jc) {
      constexpr int JT = decltype(jc)::value;
      sfor<0, 4>([&](auto rc) {
        constexpr int R = decltype(rc)::value;
        sc[JT][R] = row_bcast<(4 * JT + R) * (16 / M)>(sown);
      });
    });
    sfor<0, RT>([&](auto ic) {
      constexpr int IT = decltype(ic)::value;
      sfor<0, (IT < NT ? IT + 1 : NT)>([&](auto jc) {
        constexpr int JT = decltype(jc)::value;
#pragma unroll
        for (int r = 0; r < 4; ++r) Lt[IT][JT][r] *= sc[JT][r];
      });
    });
    if constexpr (!k16) {
      sfor<0, NT>([&](auto jc) {
        constexpr int JT = decltype(jc)::value;
#pragma unroll
        for (int r = 0; r < 4; ++r) l21[JT][r] *= sc[JT][r];
      });
    }
    if (__builtin_expect(any_bad, 0)) {
      // columns with zero / non-finite norm restart from D_jj e_j
      st_bits |= TASER_VEC_ZERO_NORM;
      sfor<0, NT>([&](auto jc) {
        constexpr int JT = decltype(jc)::value;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (act[JT][r] && sc[JT][r] == 0.f && n == 4 * r + g) Lt[JT][JT][r] = Dc[JT][r];
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
  // the last row, in the layout of the float32 path's l21 (lanes n = 0)
  if constexpr (k16) {
    sfor<0, NT>([&](auto jc) {
      constexpr int JT = decltype(jc)::value;
#pragma unroll
      for (int r = 0; r < 4; ++r) l21[JT][r] = Lt[NT][JT][r];
    });
  }

  // ---------------- slicing and outputs ----------------
  for (int j = Nm1 + lane; j < job.pad_to; j += 64) {
    job.sbar[j] = 0;
    if (job.margin) job.margin[j] = 0.f;
  }
  const int bits = skip ? (nonfinite ? TASER_VEC_NONFINITE : TASER_VEC_DEGENERATE) : st_bits;
  if (lane == 0) a.status[v] = bits;
  if (n == 0) {
    sfor<0, NT>([&](auto jc) {
      constexpr int JT = decltype(jc)::value;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = 16 * JT + 4 * r + g;
        if (j < Nm1) {
          const float x = skip ? 0.f : l21[JT][r];
          job.sbar[j] = x >= 0.f ? (int8_t)1 : (int8_t)-1;
          if (job.margin) job.margin[j] = skip ? 0.f : x / Dc[JT][r];
        }
      }
    });
  }
  if (job.L) {
    float* Lo = job.L;
    sfor<0, NT>([&](auto ic) {
      constexpr int IT = decltype(ic)::value;
      sfor<0, IT + 1>([&](auto jc) {
        constexpr int JT = decltype(jc)::value;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * IT + n, j = 16 * JT + 4 * r + g;
          if (i < Nm1 && j <= i) {
            float x = Lt[IT][JT][r];
            if (skip) x = (i == j) ? Dc[JT][r] : 0.f;
            Lo[i * (i + 1) / 2 + j] = x;
          }
        }
      });
    });
    if (n == 0) {
      sfor<0, NT>([&](auto jc) {
        constexpr int JT = decltype(jc)::value;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = 16 * JT + 4 * r + g;
          if (j < Nm1) Lo[Nm1 * (Nm1 + 1) / 2 + j] = skip ? 0.f : l21[JT][r];
        }
      });
    }
    if (lane == 0) Lo[Nm1 * (Nm1 + 1) / 2 + Nm1] = skip ? DN : l22;
  }
}

// Waves per SIMD the two-tile kernels (N - 1 <= 32) are compiled for: five
// fit in 96 VGPRs without spilling (the unconstrained build takes 102, i.e.
// four waves), and the extra wave hides more of the latency of each step's
// dependency chain.  Six would need 80 and spill.
template <int NT>
constexpr int kVecWaves = NT == 2 ? 5 : 1;
// The alternative register budgets the mixed-batch launch can select per
// size bucket (taser_mixed_launch_t.waves): eight waves per SIMD for one
// tile (64 VGPRs), four for two tiles (128, room for the scheduler), three
// for four tiles (168 instead of ~200).
template <int NT>
constexpr int kAltWaves = NT == 1 ? 8 : (NT == 2 ? 4 : 3);
template <int NT, int W>
constexpr int kMixedWaves = W ? kAltWaves<NT> : kVecWaves<NT>;

// One vector per block (uniform sizes).
template <int NT, int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kVecWaves<NT>)))
void fused_vec(FusedArgs a) {
  __shared__ __align__(16) float lds[VecLds<NT>::FLOATS];
  VecJob job;
  job.v = blockIdx.x;
  job.B = a.B; job.U = a.U; job.N = a.N; job.mod = a.mod;
  const int Nm1 = a.N - 1;
  if (a.mode == TASER_JED) {
    job.H = nullptr;
    job.y = a.y + job.v * (long long)(a.U + 1) * a.B;
    job.s0 = a.s0[job.v];
  } else {
    job.H = a.H + (job.v / a.y_per_H) * (long long)a.B * a.U;
    job.y = a.y + job.v * (long long)a.B;
    job.s0 = make_float2(1.f, 0.f);
  }
  job.sbar = a.sbar + job.v * Nm1;
  job.margin = a.margin ? a.margin + job.v * Nm1 : nullptr;
  job.L = a.L_out ? a.L_out + job.v * (long long)(a.N * (a.N + 1) / 2) : nullptr;
  job.pad_to = 0;
  vec_body<NT, P>(a, job, lds);
}

// ---------------------------------------------------------------------------
// taser_build_T for N - 1 <= 64 and U <= 32: the per-vector kernel's
// preprocessing (complex Gram on the matrix cores) writes T~ and D, then the
// Lanczos norm that the general preprocessing kernel uses gives ||T~||_2, so
// lam, tau and status follow the same definitions there and here.
template <int NT>
__global__ __launch_bounds__(64) void build_T_vec(StagedArgs a) {
  constexpr int N1 = 16 * NT;
  constexpr int NMAX = N1 + 1;
  constexpr int kSteps = spectral::lanczos_steps(NMAX, false);
  constexpr int kQ = kSteps * NMAX;
  // the packed T is dead once T~ is in Tr, and the Lanczos basis reuses it
  __shared__ __align__(16) float TQ[VecLds<NT>::TT > kQ ? VecLds<NT>::TT : kQ];
  float* T = TQ;
  float* Q = TQ;
  __shared__ float Tr[NMAX * NMAX];
  __shared__ float Dl[N1 + 1];
  __shared__ float al[kSteps], be2[kSteps];
  __shared__ float lz[spectral::lanczos_scratch_floats(NMAX)];
  const int lane = threadIdx.x;
  const long long v = blockIdx.x;
  const int N = a.N, Nm1 = N - 1;
  const bool jed = a.mode == TASER_JED;
  VecJob job{};
  job.v = v;
  job.B = a.B; job.U = a.U; job.N = N; job.mod = a.mod;
  if (jed) {
    job.H = nullptr;
    job.y = a.y + v * (long long)(a.U + 1) * a.B;
    job.s0 = a.s0[v];
  } else {
    job.H = a.H + (v / a.y_per_H) * (long long)a.B * a.U;
    job.y = a.y + v * (long long)a.B;
    job.s0 = make_float2(1.f, 0.f);
  }
  vec_build_T<NT, TASER_PREC_F32, NT == 4>(job, jed, T);

  int bad = 0, deg = 0;
  for (int e = lane; e < VecLds<NT>::TT; e += 64)
    if (!isfinite(T[e])) bad = 1;
  const bool nonfinite = or_all(bad);
  for (int k = lane; k <= N1; k += 64) {
    const bool real_k = k < Nm1 || k == N1;
    const float d = nonfinite ? 0.f : fabsf(T[tix(k, k)]);
    if (real_k && d == 0.f) deg = 1;
    Dl[k] = (d == 0.f || !real_k) ? 1.f : hsqrt(d);
  }
  const bool degenerate = !nonfinite && or_all(deg);
  __syncthreads();
  float* Ttg = a.Tt + v * (long long)N * N;
  for (int e = lane; e < N * N; e += 64) {
    const int i = e / N, j = e - i * N;
    const int pi = i < Nm1 ? i : N1, pj = j < Nm1 ? j : N1;
    const float t = nonfinite ? 0.f : T[tix(pi, pj)] * rcp(Dl[pi] * Dl[pj]);
    Tr[e] = t;
    Ttg[e] = t;
  }
  for (int k = lane; k < N; k += 64) a.D[v * N + k] = Dl[k < Nm1 ? k : N1];
  __syncthreads();
  const float lam = spectral::lanczos_norm(Tr, N, a.mod == TASER_QPSK, jed, Q, al, be2, lz);
  if (lane == 0) {
    a.lam[v] = lam;
    if (a.tau_mode == TASER_TAU_SPECTRAL) a.tau[v] = a.alpha / (lam > 0.f ? lam : 1.f);
    a.status[v] = nonfinite ? TASER_VEC_NONFINITE : (degenerate ? TASER_VEC_DEGENERATE : 0);
  }
}

// Mixed-size batch: a persistent grid walks the list of vectors of one size
// bucket that the bucketing kernel left in the workspace.
template <int NT, int P>
__global__ __launch_bounds__(64) void fused_vec_mixed(FusedArgs a, MixedArgs m, int bucket) {
  __shared__ __align__(16) float lds[VecLds<NT>::FLOATS];
  const int count = m.count[bucket];
  const int32_t* list = m.list + (long long)bucket * a.V;
  // The job's sizes and offsets are the same in every lane: moving them to
  // scalar registers keeps the sizes, loop bounds and pointers of the body
  // out of the vector registers (the loads below are vector loads).
  auto uni = [](int x) { return __builtin_amdgcn_readfirstlane(x); };
  auto uni64 = [&](long long x) {
    const unsigned lo = (unsigned)uni((int)(x & 0xffffffffll));
    const unsigned hi = (unsigned)uni((int)(x >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
  };
  for (int item = blockIdx.x; item < count; item += gridDim.x) {
    VecJob job;
    job.v = uni(list[item]);
    job.B = uni(m.Bv[job.v]); job.U = uni(m.Uv[job.v]); job.mod = uni(m.modv[job.v]);
    job.N = job.mod == TASER_QPSK ? 2 * job.U + 1 : job.U + 1;
    job.H = a.H + uni64(m.H_off[job.v]);
    job.y = a.y + uni64(m.y_off[job.v]);
    job.s0 = make_float2(1.f, 0.f);
    job.sbar = a.sbar + job.v * (long long)m.stride;
    job.margin = a.margin ? a.margin + job.v * (long long)m.stride : nullptr;
    job.L = nullptr;
    job.pad_to = m.stride;
    vec_body<NT, P>(a, job, lds);
    __syncthreads();   // the next vector reuses the LDS
  }
}

// Mixed-size batch, one workgroup per entry of the batch: workgroup i takes
// entry i of the bucket's list and those past the bucket's count exit at
// once.  Without the persistent loop the body keeps its registers to itself
// (the loop made the compiler keep loop-invariant index arithmetic live
// through every vector: 198 instead of 107 VGPRs for N-1 <= 32).
__device__ __forceinline__ VecJob mixed_job(const FusedArgs& a, const MixedArgs& m, int bucket,
                                            int item) {
  VecJob job;
  job.v = m.list[(long long)bucket * a.V + item];
  job.B = m.Bv[job.v]; job.U = m.Uv[job.v]; job.mod = m.modv[job.v];
  job.N = job.mod == TASER_QPSK ? 2 * job.U + 1 : job.U + 1;
  job.H = a.H + m.H_off[job.v];
  job.y = a.y + m.y_off[job.v];
  job.s0 = make_float2(1.f, 0.f);
  job.sbar = a.sbar + job.v * (long long)m.stride;
  job.margin = a.margin ? a.margin + job.v * (long long)m.stride : nullptr;
  job.L = nullptr;
  job.pad_to = m.stride;
  return job;
}

template <int NT, int P, int W>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kMixedWaves<NT, W>)))
void fused_vec_mixed_once(FusedArgs a, MixedArgs m, int bucket) {
  __shared__ __align__(16) float lds[VecLds<NT>::FLOATS];
  const int item = blockIdx.x;
  if (item >= m.count[bucket]) return;
  vec_body<NT, P>(a, mixed_job(a, m, bucket, item), lds);
}

// Every bucket in one launch: workgroup i takes entry i of one work queue,
// the bucket lists in the order N - 1 <= 64, <= 32, <= 16 (the longest
// problems start first and the short ones fill the tail).  The body of each
// size is compiled into the one kernel, which therefore runs with the
// registers and LDS of the largest.
template <int P>
__global__ __launch_bounds__(64) void fused_vec_mixed_all(FusedArgs a, MixedArgs m) {
  __shared__ __align__(16) float lds[VecLds<4>::FLOATS];
  const int c2 = m.count[2], c1 = m.count[1], c0 = m.count[0];
  int item = blockIdx.x;
  if (item < c2) {
    vec_body<4, P>(a, mixed_job(a, m, 2, item), lds);
  } else if ((item -= c2) < c1) {
    vec_body<2, P>(a, mixed_job(a, m, 1, item), lds);
  } else if ((item -= c1) < c0) {
    vec_body<1, P>(a, mixed_job(a, m, 0, item), lds);
  }
}

// Size bucket of a mixed-batch vector: 0 = N-1 <= 16, 1 = <= 32, 2 = <= 64,
// -1 = beyond the fused kernels.
__device__ __forceinline__ int mixed_bucket(int B, int U, int mod) {
  if (B < 1 || U < 1 || U > 32 || (mod != TASER_BPSK && mod != TASER_QPSK)) return -1;
  const int nm1 = mod == TASER_QPSK ? 2 * U : U;
  return nm1 <= 16 ? 0 : (nm1 <= 32 ? 1 : (nm1 <= 64 ? 2 : -1));
}

__device__ __forceinline__ int modv_nm1(int U, int mod, int stride) {
  const int nm1 = mod == TASER_QPSK ? 2 * U : U;
  return nm1 < 0 ? 0 : (nm1 > stride ? stride : nm1);
}

__global__ void mixed_clear(int32_t* count) {
  if (threadIdx.x < kMixedBuckets) count[threadIdx.x] = 0;
}

constexpr int kAssignThreads = 1024;

// Appends every vector to its bucket's list (order within a bucket is
// arbitrary; each vector's result does not depend on it).  Vectors no fused
// kernel covers get status TASER_VEC_UNSUPPORTED and decisions +1.
__global__ __launch_bounds__(kAssignThreads) void mixed_assign(FusedArgs a, MixedArgs m) {
  __shared__ int blk_count[kMixedBuckets];
  __shared__ int blk_base[kMixedBuckets];
  if (threadIdx.x < kMixedBuckets) blk_count[threadIdx.x] = 0;
  __syncthreads();
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  int b = -2;                                   // -2: past the end, -1: unsupported size
  if (v < a.V) {
    b = mixed_bucket(m.Bv[v], m.Uv[v], m.modv[v]);
    if (b < 0) {
      a.status[v] = TASER_VEC_UNSUPPORTED;
      const int nm1 = modv_nm1(m.Uv[v], m.modv[v], m.stride);
      for (int j = 0; j < m.stride; ++j) {
        a.sbar[v * m.stride + j] = j < nm1 ? 1 : 0;
        if (a.margin) a.margin[v * m.stride + j] = 0.f;
      }
    }
  }
  // Slots are handed out at three levels, so that the three global counters
  // see one atomic per workgroup and bucket (atomics on one address
  // serialise in L2: one per wave and bucket took 60 us for 10^5 vectors):
  // lanes of a bucket take consecutive slots after their wave's offset,
  // waves after their workgroup's offset (LDS atomics), workgroups after the
  // bucket's global count.
  const int lane = threadIdx.x & 63;
  int slot = 0;
  for (int bk = 0; bk < kMixedBuckets; ++bk) {
    const unsigned long long mask = __ballot(b == bk);
    if (mask == 0ull) continue;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    int off = 0;
    if (lane == leader) off = atomicAdd(&blk_count[bk], (int)__popcll(mask));
    off = __shfl(off, leader, 64);
    if (b == bk) slot = off + (int)__popcll(mask & ((1ull << lane) - 1ull));
  }
  __syncthreads();
  if (threadIdx.x < kMixedBuckets)
    blk_base[threadIdx.x] = blk_count[threadIdx.x] ? atomicAdd(&m.count[threadIdx.x], blk_count[threadIdx.x]) : 0;
  __syncthreads();
  if (b >= 0) m.list[(long long)b * a.V + blk_base[b] + slot] = (int32_t)v;
}

template <int NT, int W>
void launch_mixed_once(const FusedArgs& a, const MixedArgs& m, int bucket, hipStream_t s) {
  const dim3 grid(a.V), block(64);
  if (a.prec == TASER_PREC_BF16)
    hipLaunchKernelGGL((fused_vec_mixed_once<NT, TASER_PREC_BF16, W>), grid, block, 0, s, a, m, bucket);
  else if (a.prec == TASER_PREC_F16)
    hipLaunchKernelGGL((fused_vec_mixed_once<NT, TASER_PREC_F16, W>), grid, block, 0, s, a, m, bucket);
  else
    hipLaunchKernelGGL((fused_vec_mixed_once<NT, TASER_PREC_F32, W>), grid, block, 0, s, a, m, bucket);
}

// blocks > 0: a persistent grid of that many workgroups; 0: one workgroup
// per entry of the batch (the default), compiled for the default (waves 0)
// or the alternative (waves 1) register budget.
template <int NT>
bool launch_mixed_nt(const FusedArgs& a, const MixedArgs& m, int bucket, int blocks, int waves,
                     hipStream_t s) {
  const dim3 block(64);
  if (blocks > 0) {
    const dim3 grid(blocks);
    if (a.prec == TASER_PREC_BF16)
      hipLaunchKernelGGL((fused_vec_mixed<NT, TASER_PREC_BF16>), grid, block, 0, s, a, m, bucket);
    else if (a.prec == TASER_PREC_F16)
      hipLaunchKernelGGL((fused_vec_mixed<NT, TASER_PREC_F16>), grid, block, 0, s, a, m, bucket);
    else
      hipLaunchKernelGGL((fused_vec_mixed<NT, TASER_PREC_F32>), grid, block, 0, s, a, m, bucket);
  } else if (waves) {
    launch_mixed_once<NT, 1>(a, m, bucket, s);
  } else {
    launch_mixed_once<NT, 0>(a, m, bucket, s);
  }
  return true;
}

template <int NT>
bool launch_vec_nt(const FusedArgs& a, hipStream_t s) {
  const dim3 grid(a.V), block(64);
  if (a.prec == TASER_PREC_BF16)
    hipLaunchKernelGGL((fused_vec<NT, TASER_PREC_BF16>), grid, block, 0, s, a);
  else if (a.prec == TASER_PREC_F16)
    hipLaunchKernelGGL((fused_vec<NT, TASER_PREC_F16>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((fused_vec<NT, TASER_PREC_F32>), grid, block, 0, s, a);
  return true;
}

}  // namespace

size_t mixed_workspace_bytes(int V) {
  return 256 + (size_t)kMixedBuckets * (size_t)V * sizeof(int32_t);
}

namespace {
// Two side streams and their fork / join events per device, created on first
// use (default priority, non-blocking) and kept until the process ends.  The
// mutex also covers the launch sequence that uses them, so calls from
// several host threads do not re-record an event between its record and
// the waits on it.
constexpr int kForkDevices = 64;
struct ForkJoin {
  hipStream_t side[2];
  hipEvent_t fork, join[2];
  bool ready;
};
ForkJoin g_fork[kForkDevices];
std::mutex g_fork_mu;

hipError_t fork_join_for_device(ForkJoin** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kForkDevices) return hipErrorInvalidDevice;
  ForkJoin& f = g_fork[dev];
  if (!f.ready) {
    for (int i = 0; i < 2; ++i) {
      if ((e = hipStreamCreateWithFlags(&f.side[i], hipStreamNonBlocking)) != hipSuccess) return e;
      if ((e = hipEventCreateWithFlags(&f.join[i], hipEventDisableTiming)) != hipSuccess) return e;
    }
    if ((e = hipEventCreateWithFlags(&f.fork, hipEventDisableTiming)) != hipSuccess) return e;
    f.ready = true;
  }
  *out = &f;
  return hipSuccess;
}
}  // namespace

hipError_t launch_mixed(const FusedArgs& a, const MixedArgs& m, const taser_mixed_launch_t* launch,
                        hipStream_t s) {
  hipLaunchKernelGGL(mixed_clear, dim3(1), dim3(64), 0, s, m.count);
  hipLaunchKernelGGL(mixed_assign, dim3((a.V + kAssignThreads - 1) / kAssignThreads), dim3(kAssignThreads), 0,
                     s, a, m);
  if (launch && launch->single_launch) {
    const dim3 grid(a.V), block(64);
    if (a.prec == TASER_PREC_BF16)
      hipLaunchKernelGGL(fused_vec_mixed_all<TASER_PREC_BF16>, grid, block, 0, s, a, m);
    else if (a.prec == TASER_PREC_F16)
      hipLaunchKernelGGL(fused_vec_mixed_all<TASER_PREC_F16>, grid, block, 0, s, a, m);
    else
      hipLaunchKernelGGL(fused_vec_mixed_all<TASER_PREC_F32>, grid, block, 0, s, a, m);
    return hipGetLastError();
  }
  auto bucket = [&](int b, hipStream_t st) {
    const int g = launch ? launch->blocks[b] : 0;
    const int w = launch ? launch->waves[b] : 0;
    if (b == 0) launch_mixed_nt<1>(a, m, b, g, w, st);
    if (b == 1) launch_mixed_nt<2>(a, m, b, g, w, st);
    if (b == 2) launch_mixed_nt<4>(a, m, b, g, w, st);
  };
  if (!(launch && launch->concurrent)) {
    for (int b = 0; b < kMixedBuckets; ++b) bucket(b, s);
    return hipGetLastError();
  }
  // the three bucket kernels on three streams, so that the GPU can place
  // waves of one bucket beside those of another (the largest problems'
  // register budget leaves room on each SIMD for the small ones)
  std::lock_guard<std::mutex> lock(g_fork_mu);
  ForkJoin* f = nullptr;
  hipError_t e = fork_join_for_device(&f);
  if (e != hipSuccess) return e;
  if ((e = hipEventRecord(f->fork, s)) != hipSuccess) return e;
  for (int i = 0; i < 2; ++i)
    if ((e = hipStreamWaitEvent(f->side[i], f->fork, 0)) != hipSuccess) return e;
  bucket(2, s);
  bucket(1, f->side[0]);
  bucket(0, f->side[1]);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int i = 0; i < 2; ++i) {
    if ((e = hipEventRecord(f->join[i], f->side[i])) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s, f->join[i], 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

int fused_vec_tiles(const FusedArgs& a) {
  const int nm1 = a.N - 1;
  if (a.U > 32) return 0;                       // Gram entries per lane and staging bound
  if (a.B < 1) return 0;
  if (a.mode == TASER_JED && a.y_per_H != 1) return 0;
  if (nm1 <= 16) return 1;
  if (nm1 <= 32) return 2;
  if (nm1 <= 64) return 4;
  return 0;
}

hipError_t launch_fused_vec(const FusedArgs& a, hipStream_t s) {
  switch (fused_vec_tiles(a)) {
    case 1: launch_vec_nt<1>(a, s); break;
    case 2: launch_vec_nt<2>(a, s); break;
    case 4: launch_vec_nt<4>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int build_T_vec_tiles(const StagedArgs& a) {
  if (a.U > 32 || a.B < 1) return 0;
  if (a.mode == TASER_JED && a.y_per_H != 1) return 0;
  const int nm1 = a.N - 1;
  return nm1 <= 16 ? 1 : nm1 <= 32 ? 2 : nm1 <= 64 ? 4 : 0;
}

hipError_t launch_build_T_vec(const StagedArgs& a, hipStream_t s) {
  switch (build_T_vec_tiles(a)) {
    case 1: hipLaunchKernelGGL(build_T_vec<1>, dim3(a.V), dim3(64), 0, s, a); break;
    case 2: hipLaunchKernelGGL(build_T_vec<2>, dim3(a.V), dim3(64), 0, s, a); break;
    case 4: hipLaunchKernelGGL(build_T_vec<4>, dim3(a.V), dim3(64), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace taser
