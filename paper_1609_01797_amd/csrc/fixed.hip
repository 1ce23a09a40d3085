// Algorithm 1 in the 14-bit fixed-point arithmetic of the paper's hardware
// (Section IV-C): L~ and V with 8 fraction bits, 7 in the bottom row, the
// held L~_NN with 5, and the column scale from a 2^11-word inverse-square-
// root table with 13 fraction bits.  Where the paper leaves the arithmetic
// open, the readings are: 14-bit two's complement words that saturate;
// T^ = 2 tau T~ with 12 fraction bits; D_kk with the 8 fraction bits of the
// diagonal element it initialises (D_NN with 5); exact accumulation of a
// processing element's products with one rounding when V_ij is stored
// (round to nearest, ties upwards); exact squared column norms with 16
// fraction bits; the table indexed by the top 11 bits of the squared norm
// after an even normalising shift, entry i holding the integer nearest to
// 2^13 / sqrt((i + 1/2) / 2^10); a scale factor D_jj / ||v_j|| with 11
// fraction bits; a zero column reset to D_jj e_j.
//
// One wave per vector: lane j owns column j.  It holds column j of T^ in
// registers and forms column j of V row by row, reading row i of L~ from LDS
// as a broadcast; its column norm, scale factor and prox are lane-local, and
// it writes its column of the new L~ back to LDS for the next iteration.
#include "taser_internal.h"

namespace taser {
namespace {

constexpr int kFL = 8, kFB = 7, kFNN = 5, kFT = 12, kFC = 11;
constexpr int kWMin = -8192, kWMax = 8191;

// The inverse-square-root table, computed at compile time with integer
// arithmetic only: r is the integer nearest to 2^18 / sqrt(i + 1/2) exactly
// when (2r - 1)^2 (2i + 1) <= 2^39 < (2r + 1)^2 (2i + 1) (the bound is never
// met with equality: the left sides are odd), so the entry is the smallest r
// with (2r + 1)^2 (2i + 1) > 2^39.  Entries below 512 are never indexed.
struct RsqrtTable {
  short v[2048];
};
constexpr RsqrtTable make_rsqrt_table() {
  RsqrtTable t{};
  for (int i = 512; i < 2048; ++i) {
    const unsigned long long m = 2ull * (unsigned long long)i + 1ull, lim = 1ull << 39;
    unsigned long long lo = 0, hi = 1ull << 14;
    while (lo < hi) {
      const unsigned long long mid = (lo + hi) / 2;
      if ((2 * mid + 1) * (2 * mid + 1) * m > lim) hi = mid;
      else lo = mid + 1;
    }
    t.v[i] = (short)lo;
  }
  return t;
}
__constant__ RsqrtTable kRsqrt = make_rsqrt_table();

__device__ __forceinline__ int sat14(long long x) {
  return x < kWMin ? kWMin : (x > kWMax ? kWMax : (int)x);
}

// floor(x / 2^s + 1/2), s >= 1
__device__ __forceinline__ long long round_shift(long long x, int s) {
  return (x + (1ll << (s - 1))) >> s;
}

// D_jj / ||v_j|| with 11 fraction bits from the squared norm q > 0 (16
// fraction bits) and D_jj (8 fraction bits): q = idx 2^s with s even gives
// 1/sqrt(q 2^-16) = table[idx] 2^(-10 - s/2), so the factor in units of
// 2^-11 is d table[idx] 2^(-7 - s/2).
__device__ __forceinline__ int scale_factor(long long q, int d) {
  const int p = 64 - __clzll((unsigned long long)q);   // bit length, >= 1
  int s = p - 11;
  s += s & 1;
  const int idx = (int)(s >= 0 ? (q >> s) : (q << (-s)));
  const int shift = 7 + s / 2;                         // >= 2: q >= 1 gives s >= -10
  const long long v = round_shift((long long)d * (long long)kRsqrt.v[idx], shift);
  return v < 0 ? 0 : (v > kWMax ? kWMax : (int)v);
}

// Preprocessing outputs -> words: T^ = 2 tau T~ (12 fraction bits), D_kk
// (8; D_NN 5), round to nearest with ties upwards, saturating.  2 tau T~ is
// one float32 product (never contracted into a later add, so both kernels
// that quantise get the same value); scaling by 2^F is exact, and so is
// floor(x + 1/2) in the 14-bit range (larger values saturate either way).
__device__ __forceinline__ int16_t quantize(float x, int frac) {
  const float s = floorf(__fadd_rn(ldexpf(x, frac), 0.5f));
  return (int16_t)(s < (float)kWMin ? kWMin : (s > (float)kWMax ? kWMax : (int)s));
}
__device__ __forceinline__ int16_t quantize_That(float two_tau, float t) {
  return quantize(__fmul_rn(two_tau, t), kFT);
}

// Inputs are words (That, D) or, when Tt is set, the float32 preprocessing
// outputs T~, D, tau, quantised here exactly as fixed_quantize_kernel does;
// the output L~ is words (L) or their real values (Lf).
template <int NP>
__global__ __launch_bounds__(64) void fixed_solve_kernel(FixedArgs a) {
  __shared__ int Ls[NP][NP];       // L~ (rows in their own formats; L~_NN aligned to 7 bits)
  const int j = threadIdx.x;
  const long long v = blockIdx.x;
  const int N = a.N;
  const bool col = j < N;
  const int jc = col ? j : 0;      // an in-range column for lanes past N (their results are dropped)
  int Tc[NP];                      // column j of T^
  int dj, lnn;
  if (a.Tt) {
    const float* Tv = a.Tt + v * (long long)N * N;
    const float t2 = 2.f * a.tau[v];
#pragma unroll
    for (int k = 0; k < NP; ++k) Tc[k] = (col && k < N) ? (int)quantize_That(t2, Tv[(long long)k * N + j]) : 0;
    dj = col ? (int)quantize(a.Df[v * N + j], j == N - 1 ? kFNN : kFL) : 0;
    lnn = (int)quantize(a.Df[v * N + N - 1], kFNN);
  } else {
    const int16_t* Tv = a.That + v * (long long)N * N;
#pragma unroll
    for (int k = 0; k < NP; ++k) Tc[k] = (col && k < N) ? (int)Tv[(long long)k * N + j] : 0;
    dj = col ? (int)a.D[v * N + j] : 0;
    lnn = (int)a.D[v * N + N - 1];
  }
  const int st_in = a.status[v];
  const bool skip = (st_in & (TASER_VEC_DEGENERATE | TASER_VEC_NONFINITE)) != 0;
  // L~(0) = D
  if (j < NP)
    for (int i = 0; i < NP; ++i) Ls[i][j] = (i == j && j < N - 1) ? dj : 0;
  __syncthreads();
  if (j == 0) Ls[N - 1][N - 1] = lnn << (kFB - kFNN);
  __syncthreads();
  int bits = 0;
  const int iters = skip ? 0 : a.t_max;
  for (int t = 0; t < iters; ++t) {
    // V = L~ - tril(L~ T^): column j, rows i >= j; row i of L~ is read
    // whole (a broadcast) before any lane writes
    int Vc[NP];
    long long q = 0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      Vc[i] = 0;
      if (i < N) {
        long long acc = (long long)Ls[i][jc] << kFT;
#pragma unroll
        for (int k = 0; k <= i; ++k) acc -= (long long)Ls[i][k] * (long long)Tc[k];
        const int x = (j <= i) ? sat14(round_shift(acc, kFT)) : 0;
        Vc[i] = x;
        // squared column norm, 16 fraction bits (bottom row aligned by 2^2)
        const long long x2 = (long long)x * (long long)x;
        q += (i == N - 1) ? (x2 << (2 * (kFL - kFB))) : x2;
      }
    }
    __syncthreads();               // every lane has read L~ before it is overwritten
    if (col && j < N - 1) {
      if (q == 0) {
        bits |= TASER_VEC_ZERO_NORM;
#pragma unroll
        for (int i = 0; i < NP; ++i)
          if (i < N) Ls[i][j] = (i == j) ? dj : 0;
      } else {
        const int c = scale_factor(q, dj);
#pragma unroll
        for (int i = 0; i < NP; ++i)
          if (i < N) Ls[i][j] = sat14(round_shift((long long)Vc[i] * (long long)c, kFC));
      }
    }
    __syncthreads();
  }
  // outputs: packed words (row N with its 7-bit values and L~_NN's 5-bit
  // register value), decisions sign(L~_Nk), status
  if (col) {
    const long long o = v * (long long)(N * (N + 1) / 2);
    for (int i = j; i < N; ++i) {
      const int w = (i == N - 1 && j == N - 1) ? lnn : Ls[i][j];
      if (a.L) a.L[o + i * (i + 1) / 2 + j] = (int16_t)w;
      if (a.Lf) {
        const int f = i < N - 1 ? kFL : (j < N - 1 ? kFB : kFNN);
        a.Lf[o + i * (i + 1) / 2 + j] = ldexpf((float)w, -f);   // exact
      }
    }
    if (j < N - 1 && a.sbar) a.sbar[v * (long long)(N - 1) + j] = Ls[N - 1][j] >= 0 ? 1 : -1;
  }
  const unsigned long long any = __ballot(bits != 0);
  if (j == 0) a.status[v] = skip ? st_in : (st_in | (any ? TASER_VEC_ZERO_NORM : 0));
}

__global__ __launch_bounds__(256) void fixed_quantize_kernel(FixedArgs a, const float* __restrict__ Tt,
                                                             const float* __restrict__ D,
                                                             const float* __restrict__ tau,
                                                             int16_t* __restrict__ That,
                                                             int16_t* __restrict__ Dq) {
  const long long v = blockIdx.y;
  const int N = a.N;
  const float t2 = 2.f * tau[v];
  for (int e = blockIdx.x * 256 + threadIdx.x; e < N * N; e += gridDim.x * 256)
    That[v * N * N + e] = quantize_That(t2, Tt[v * N * N + e]);
  if (blockIdx.x == 0)
    for (int k = threadIdx.x; k < N; k += 256)
      Dq[v * N + k] = quantize(D[v * N + k], k == N - 1 ? kFNN : kFL);
}

template <typename F>
hipError_t dispatch_np(int N, F&& f) {
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

}  // namespace

hipError_t launch_fixed_quantize(const FixedArgs& a, const float* Tt, const float* D,
                                 const float* tau, int16_t* That, int16_t* Dq, hipStream_t s) {
  const int per = (a.N * a.N + 255) / 256;
  // grid.y indexes vectors: at most 65,535 per launch
  for (long long v0 = 0; v0 < a.V; v0 += 65535) {
    const int n = (int)(a.V - v0 < 65535 ? a.V - v0 : 65535);
    const long long o = v0;
    hipLaunchKernelGGL(fixed_quantize_kernel, dim3(per, n), dim3(256), 0, s, a, Tt + o * a.N * a.N,
                       D + o * a.N, tau + o, That + o * a.N * a.N, Dq + o * a.N);
  }
  return hipGetLastError();
}

hipError_t launch_fixed_solve(const FixedArgs& a, hipStream_t s) {
  return dispatch_np(a.N, [&](auto np) {
    constexpr int NP = decltype(np)::value;
    hipLaunchKernelGGL(fixed_solve_kernel<NP>, dim3(a.V), dim3(64), 0, s, a);
    return hipGetLastError();
  });
}

}  // namespace taser
