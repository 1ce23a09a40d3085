/*
 * taser.h -- C ABI of libtaser.so, a batched TASER detector for AMD MI355X
 * (gfx950).
 *
 * TASER (Triangular Approximate SEmidefinite Relaxation; Castaneda,
 * Goldstein and Studer, arXiv:1609.01797) detects BPSK/QPSK symbols in
 * coherent MU-MIMO systems (Section II-A) and jointly estimates the channel
 * and detects the data in SIMO block-fading systems (Section II-B).  Both
 * problems become  min over s~ in {-1,+1}^N of s~^T T s~  (eq. (2), eq. (5)),
 * which Algorithm 1 solves approximately with preconditioned forward-backward
 * splitting on a lower-triangular factor L~ (Sections III-A to III-D).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every data pointer is a DEVICE pointer owned by the caller.  The library
 *    never allocates, never frees and keeps no per-call state.
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream).  Outputs are valid once the stream has reached the call.
 *  - Argument, shape and support errors are returned synchronously, before
 *    anything is launched, and then no output is written.  A failed HIP call
 *    or launch returns TASER_ERR_DEVICE.
 *  - Numerical conditions never abort: they set per-vector status bits
 *    (TASER_VEC_*) in an int32 status[V] array.
 *  - Complex numbers are interleaved float32 pairs (re, im), i.e. the
 *    memory layout of C99 float complex / numpy complex64.
 *  - Real vector index s~ = [Re s_1..Re s_U, Im s_1..Im s_U, 1] for QPSK
 *    and [s_1..s_U, 1] for BPSK (Section II-A); N = 2U+1 or U+1.
 *  - Lower-triangular matrices are packed row by row:
 *    element (i, j), j <= i, sits at i*(i+1)/2 + j.
 *
 * Readings of the paper that change results (all switchable where noted):
 *  - The prox of Section III-C normalises each COLUMN k of L~ to norm D_kk.
 *  - D_kk = sqrt(|T_kk|): the joint-detection T of eq. (5) is negative
 *    semidefinite, so its diagonal is negative.
 *  - L~_NN is held at D_NN (the hardware of Section IV-C keeps it constant);
 *    TASER_FLAG_LITERAL_LAST normalises it like every other column instead.
 *  - sign(0) = +1 when slicing.
 *  - A column whose norm is zero or non-finite is reset to D_kk e_k.
 */
#ifndef TASER_H
#define TASER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TASER_ABI_VERSION 3
#define TASER_MAX_N 129          /* largest problem size N the library accepts */
#define TASER_MAX_VECTORS (1 << 30) /* largest num_vectors any entry point accepts
                                       (kernel indices stay within 32 bits) */

typedef enum {
  TASER_OK = 0,
  TASER_ERR_ARG = -1,            /* null pointer, bad enum, bad alpha / t_max */
  TASER_ERR_SHAPE = -2,          /* sizes out of range or inconsistent */
  TASER_ERR_UNSUPPORTED = -3,    /* valid request the library does not implement */
  TASER_ERR_WORKSPACE = -4,      /* workspace pointer NULL or smaller than required */
  TASER_ERR_DEVICE = -5          /* a HIP call or kernel launch failed */
} taser_status_t;

enum { TASER_BPSK = 1, TASER_QPSK = 2 };
enum { TASER_COHERENT = 0, TASER_JED = 1 };
/* Arithmetic of the main loop.  F32 / BF16 / F16 select the operands of the
   L~ T~ products; norms, rsqrt, the preconditioner and the master copy of L~
   are float32 in those modes.  FIXED14 runs the whole loop in the 14-bit
   fixed-point arithmetic of the paper's hardware (Section IV-C; see
   taser_fixed_solve) and is accepted by taser_solve only. */
enum { TASER_PREC_F32 = 0, TASER_PREC_BF16 = 1, TASER_PREC_F16 = 2, TASER_PREC_FIXED14 = 3 };
enum { TASER_TAU_SPECTRAL = 0,   /* tau = alpha / ||T~||_2 (Algorithm 1 inputs) */
       TASER_TAU_GIVEN = 1 };    /* tau[v] supplied by the caller */

#define TASER_FLAG_LITERAL_LAST 1 /* normalise column N too (L~_NN = D_NN sign V_NN) */

/* per-vector status bits */
#define TASER_VEC_DEGENERATE 1   /* some T_kk == 0: no iterations; L~ = D */
#define TASER_VEC_NONFINITE  2   /* NaN/Inf reached T: no iterations; L~ = D */
#define TASER_VEC_ZERO_NORM  4   /* a prox column had zero norm and was reset */
#define TASER_VEC_VNN_NONPOS 8   /* V_NN <= 0 occurred in some iteration */
#define TASER_VEC_UNSUPPORTED 16 /* mixed batch: no fused kernel for this size; decisions +1 */

typedef struct {
  int32_t num_vectors;  /* 0 <= V <= TASER_MAX_VECTORS: received vectors
                           (coherent) or blocks (JED) */
  int32_t B;            /* receive antennas, >= 1 */
  int32_t U;            /* coherent: users; JED: K, the data slots after the pilot */
  int32_t mod;          /* TASER_BPSK or TASER_QPSK */
  int32_t mode;         /* TASER_COHERENT or TASER_JED */
  int32_t prec;         /* TASER_PREC_* */
  int32_t tau_mode;     /* TASER_TAU_* */
  int32_t y_per_H;      /* coherent: consecutive vectors sharing one H (>= 1,
                           divides num_vectors); JED: must be 1 */
  int32_t t_max;        /* iterations, 0 <= t_max <= 100000 */
  int32_t flags;        /* TASER_FLAG_* */
  float alpha;          /* 0 < alpha < 1 when tau_mode == TASER_TAU_SPECTRAL */
} taser_desc_t;

/* Version of this ABI (TASER_ABI_VERSION of the built library). */
int taser_abi_version(void);

/* Testing aid for callers' error paths: the next `count` calls of entry
   points that launch device work return TASER_ERR_DEVICE after their
   argument checks and before they launch anything (count = 0 clears it).
   Host-only and process-wide; argument and shape errors still take
   precedence.  Errors: TASER_ERR_ARG for count < 0. */
taser_status_t taser_debug_inject_device_error(int32_t count);

/* Static text for a taser_status_t value. */
const char* taser_status_string(int status);

/* Problem size N of the real-valued reformulation (Section II): 2U+1 for
   QPSK, U+1 for BPSK; -1 for an invalid modulation or U < 1. */
int taser_problem_size(int U, int mod);

/* Host-only validation of a descriptor (no device work): TASER_OK or the
   error the entry points would return for it. */
taser_status_t taser_check_desc(const taser_desc_t* desc);

/* Preprocessing: build T (eq. (2) or eq. (5)) and precondition it
   (Section III-C), then form the step size of Algorithm 1.
   Inputs
     coherent: H complex64 [V/y_per_H][B][U] row-major (vector v uses
               H[v / y_per_H]); y complex64 [V][B]; s0 ignored (may be NULL).
     JED:      H ignored (may be NULL); y holds Y, complex64 [V][U+1][B]
               slot-major (y[v][k][b] = antenna b in slot k; slot 0 carries
               the pilot); s0 complex64 [V], the known first entry s_0 of
               the paper's s.
   Outputs (float32)
     Tt   [V][N][N]  T~ = D^-1 T D^-1, full symmetric matrix
     D    [V][N]     D_kk = sqrt(|T_kk|)
     lam  [V]        ||T~||_2 (largest |eigenvalue|, Lanczos in float32)
     tau  [V]        written with alpha/lam when tau_mode == SPECTRAL;
                     left untouched (an input of taser_solve) when GIVEN
     status [V]      TASER_VEC_DEGENERATE / TASER_VEC_NONFINITE or 0 */
taser_status_t taser_build_T(const taser_desc_t* desc, const void* H, const void* y,
                             const void* s0, float* Tt, float* D, float* lam, float* tau,
                             int32_t* status, void* stream);

/* Algorithm 1, initialisation and main loop (Section III-D):
   L~(0) = D; t_max times  V = L~ - tril(2 tau L~ T~),  L~ = prox(V).
   Inputs: Tt [V][N][N], D [V][N], tau [V] (float32), status [V] from
   taser_build_T (vectors flagged DEGENERATE or NONFINITE run no iterations
   and get L~ = D).  Output: L [V][N(N+1)/2] packed float32; status gains
   TASER_VEC_ZERO_NORM / TASER_VEC_VNN_NONPOS bits.  desc->prec: TASER_PREC_F32,
   or TASER_PREC_FIXED14 (N <= 64): T^ = 2 tau T~ and D are quantised as
   taser_fixed_quantize does, the loop runs as taser_fixed_solve, and L holds
   the exact real values of the resulting words (VNN_NONPOS is not
   reported: the hardware has no element for V_NN).  Other precisions return
   TASER_ERR_UNSUPPORTED. */
taser_status_t taser_solve(const taser_desc_t* desc, const float* Tt, const float* D,
                           const float* tau, float* L, int32_t* status, void* stream);

/* ---- Reference detectors (Section V-A) ----------------------------------

   The detectors the paper compares TASER with, on the real-valued model of
   Section II-A (ybar = Hbar sbar + nbar, sbar in {-1,+1}^M, M = N - 1),
   coherent requests only (desc->mode = TASER_COHERENT; B, U, mod, y_per_H,
   num_vectors as for taser_run; t_max, prec, tau_mode and alpha unused):
     TASER_REF_MF     the matched filter: sign(Hbar^T ybar) (Algorithm 1
                      after one iteration has the same signs);
     TASER_REF_MMSE   linear MMSE with unit symbol energy per real dimension:
                      sign((Hbar^T Hbar + (n0/2) I)^-1 Hbar^T ybar), n0 >= 0
                      the complex noise variance N0 of y = Hs + n;
     TASER_REF_ML     exhaustive ML of eq. (1), argmin ||ybar - Hbar s||^2
                      over all 2^M candidates, M <= 20 (ties: the candidate
                      with the smaller bit pattern, bit j set for s_j = -1);
     TASER_REF_KBEST  K-best breadth-first search (1 <= K <= 16) after
                      Hbar^T Hbar = R^T R: from the last real dimension to
                      the first each surviving path is extended by +1 and -1
                      and the K of smallest partial distance survive (ties:
                      the earlier candidate, path rank first, +1 first).
   Float32 arithmetic.  Out: sbar int8 [V][M] in s~ order (sign(0) = +1);
   soft (or NULL): MF / MMSE the estimates [V][M] before slicing, ML /
   K-best the residual ||ybar - Hbar shat||^2 [V].  A singular Hbar^T Hbar
   (K-best with M > 2B, or a zero channel column) does not fault: pivots
   are clamped to the smallest normal float.  Errors: those of
   taser_check_desc, TASER_ERR_ARG (kind, K, n0 < 0 or non-finite, NULL
   pointers), TASER_ERR_UNSUPPORTED (JED, M > 64, ML with M > 20). */
enum { TASER_REF_MF = 0, TASER_REF_MMSE = 1, TASER_REF_ML = 2, TASER_REF_KBEST = 3 };
taser_status_t taser_reference_detect(const taser_desc_t* desc, int32_t kind, int32_t K, float n0,
                                      const void* H, const void* y, int8_t* sbar, float* soft,
                                      void* stream);

/* ---- Exact semidefinite relaxation (eq. (7)) -----------------------------

   The detector TASER approximates: S^ = argmin Tr(T S) subject to
   diag(S) = 1 and S positive semidefinite, then (Section II-C) the signs
   of the leading eigenvector of S^, oriented so that its last entry (the
   fixed entry of s~) is non-negative; sign(0) = +1.  Both modes, 2 <= N <=
   65 (desc: mode, B, U, mod, num_vectors as for taser_build_T; t_max,
   prec, tau_mode, alpha unused).  Solved per vector in float64 by a
   primal-dual interior-point method (HKM direction, adaptive centring,
   backtracked steps at 0.95 of the boundary) until the duality gap is
   below 1e-9 max(1, |Tr(C X)|) in the scaled units C = T / max|T_ij|, a
   factorisation fails, the gap stalls below 1e-6 max(1, |Tr(C X)|), or
   100 iterations.
   In: Tt [V][N][N] and D [V][N] (float32) as taser_build_T writes them
       (T = D T~ D), or D = NULL and Tt holding T itself; status [V] or
       NULL (vectors with a nonzero entry are skipped: sbar = +1, X = I,
       zeros).
   Out: sbar int8 [V][N-1]; each of the rest may be NULL: objective [V] =
       Tr(T X), gap [V] = Tr(T X) - sum(y) >= 0 (the duality gap, units of
       T), X [V][N][N] (the final primal iterate), all float64;
       iterations [V].
   Errors: those of taser_check_desc, TASER_ERR_ARG (NULL Tt or sbar with
   V > 0), TASER_ERR_UNSUPPORTED (N > 65). */
taser_status_t taser_sdr_detect(const taser_desc_t* desc, const float* Tt, const float* D,
                                const int32_t* status, int8_t* sbar, double* objective, double* gap,
                                double* X, int32_t* iterations, void* stream);

/* ---- Fixed-point mode (Section IV-C) ----------------------------------

   Algorithm 1 in the 14-bit fixed-point arithmetic of the paper's systolic
   array.  A word is a 14-bit two's complement integer w with value
   w 2^-F; words saturate at [-8192, 8191].  Fraction bits F, as the paper
   gives them: 8 for L~ and V in rows 1..N-1, 7 in row N (the bottom row of
   the array), 5 for L~_NN (held constant at D_NN).  Readings where the
   paper is silent: T^ = 2 tau T~ with 12 fraction bits, D_kk with 8 (D_NN
   with 5); each V_ij is its exact sum of products rounded once (to nearest,
   ties upwards); column norms are exact with 16 fraction bits; the inverse
   square root comes from a 2^11-entry table of 14-bit words with 13
   fraction bits (entry i: the integer nearest to 2^13/sqrt((i+1/2)/2^10)),
   indexed by the top 11 bits of the squared norm after an even normalising
   shift; the scale factor D_jj/||v_j|| has 11 fraction bits.  N <= 64;
   larger problems return TASER_ERR_UNSUPPORTED.

   taser_fixed_quantize: the preprocessing outputs of taser_build_T (Tt
   [V][N][N], D [V][N], tau [V], float32) to words: That int16 [V][N][N],
   Dq int16 [V][N].  2 tau T~ is formed as one float32 product.
   taser_fixed_solve: L~(0) = D, t_max fixed-point iterations and slicing.
   In: That, Dq (words), status [V] from taser_build_T (DEGENERATE or
   NONFINITE vectors run no iterations).  Out: L int16 [V][N(N+1)/2] packed
   rows of words (row N holds 7-bit words and the 5-bit L~_NN); sbar int8
   [V][N-1] = sign(L~_Nk) with sign(0) = +1, or NULL; status gains
   TASER_VEC_ZERO_NORM when a column of V was zero (reset to D_jj e_j).
   All arrays are device memory owned by the caller; errors: those of
   taser_check_desc, TASER_ERR_ARG (NULL pointers), TASER_ERR_UNSUPPORTED. */
taser_status_t taser_fixed_quantize(const taser_desc_t* desc, const float* Tt, const float* D,
                                    const float* tau, int16_t* That, int16_t* Dq, void* stream);
taser_status_t taser_fixed_solve(const taser_desc_t* desc, const int16_t* That, const int16_t* Dq,
                                 int16_t* L, int8_t* sbar, int32_t* status, void* stream);

/* Algorithm 1 output: sbar_k = sign(L~_{N,k}) for k = 1..N-1 (sign(0) = +1),
   int8 sbar [V][N-1] in s~ order; margin [V][N-1] float32 = L~_{N,k}/D_kk
   (the last row of L = L~ D^-1, in [-1, 1]), or NULL. */
taser_status_t taser_detect(const taser_desc_t* desc, const float* L, const float* D,
                            int8_t* sbar, float* margin, void* stream);

/* Channel estimate of joint estimation and detection (Section II-B, eq. (4)):
   h = Y [s0; s_r] for every block, h_b = sum_k Y[k][b] s_k, where s_k (k >= 1)
   are the detected data symbols read from sbar (QPSK s_k = sbar[k-1] +
   j sbar[K+k-1], BPSK s_k = sbar[k-1]).  desc: a JED descriptor (U = K data
   slots).  Y: complex64 [V][K+1][B] slot-major, s0: complex64 [V] pilots,
   sbar: int8 [V][N-1] as written by taser_run / taser_detect, h: complex64
   [V][B] (out); device memory owned by the caller.  Errors: those of
   taser_check_desc, TASER_ERR_ARG (not JED, NULL pointers). */
taser_status_t taser_jed_channel(const taser_desc_t* desc, const void* Y, const void* s0,
                                 const int8_t* sbar, void* h, void* stream);

/* Device workspace (bytes) that taser_run needs for this descriptor, written
   to *bytes: 4,352 bytes per 16 vectors on the group path, 0 on the
   per-vector path.  Host-only; returns the same errors as taser_run would
   for the descriptor (TASER_ERR_UNSUPPORTED for a shape neither path
   covers). */
taser_status_t taser_workspace_size(const taser_desc_t* desc, size_t* bytes);

/* The whole detector (build T, precondition, step size, t_max iterations,
   slicing) in one call, with T~ and L~ kept on chip.  Two kernel families
   serve it, chosen from the descriptor:
     group path: coherent QPSK with U = 16 (N = 33) and y_per_H a multiple
       of 16.  Two kernels on `stream`: a preprocessing kernel that leaves
       each channel group's preconditioned G~, border c~, D and tau in the
       workspace, and a solve kernel that keeps L~ in registers (one wave
       per 16 vectors of a channel).  Workspace: taser_workspace_size()
       bytes.
     per-vector path: every other request with N - 1 <= 64 and U <= 32,
       coherent (any y_per_H) or JED, BPSK or QPSK.  One kernel, one wave
       per vector; it needs no workspace (taser_workspace_size() gives 0 and
       ws may be NULL).
   Other requests (U > 32 or N - 1 > 64) return TASER_ERR_UNSUPPORTED: use
   taser_build_T / taser_solve / taser_detect, which cover N <= TASER_MAX_N.
   Same inputs as taser_build_T; tau_in [V] is read when tau_mode == GIVEN
   (else may be NULL).  ws: device buffer of at least
   taser_workspace_size() bytes owned by the caller (contents on entry are
   ignored; calls that share a workspace must not overlap).
   Outputs: sbar int8 [V][N-1]; margin float32 [V][N-1] or NULL; status [V];
   L_out [V][N(N+1)/2] float32 or NULL (written only when non-NULL). */
taser_status_t taser_run(const taser_desc_t* desc, const void* H, const void* y,
                         const void* s0, const float* tau_in, int8_t* sbar, float* margin,
                         int32_t* status, float* L_out, void* ws, size_t ws_bytes,
                         void* stream);

/* taser_run without a workspace argument, for callers that cannot allocate
   device memory (code under HIP graph capture, tight serving loops,
   harnesses that forbid allocation).  The group path keeps its per-group
   state in a device array inside the library (TASER_STATIC_MAX_VECTORS
   vectors, 17 MiB, held on each device the library runs on until the
   process ends); the per-vector path needs no state.  Same arguments,
   kernels and results as taser_run.  The call allocates and frees nothing.
   Calls on one device share that array: calls that overlap on one device
   (on different streams, or from several threads) race and must not be
   issued.  Errors: those of taser_run; TASER_ERR_WORKSPACE for a group-path
   request of more than TASER_STATIC_MAX_VECTORS vectors. */
#define TASER_STATIC_MAX_VECTORS 65536
taser_status_t taser_run_static(const taser_desc_t* desc, const void* H, const void* y,
                                const void* s0, const float* tau_in, int8_t* sbar, float* margin,
                                int32_t* status, float* L_out, void* stream);

/* The two stages of taser_run, for callers that time or schedule them
   separately.  taser_run_prep: T assembly, Jacobi preconditioning and the
   step size (Section II, Section III-C), leaving each group's state in `ws`
   and writing status [V].  taser_run_solve: t_max iterations of Algorithm 1
   and slicing from that state; the descriptor must equal the one given to
   taser_run_prep (except prec, which selects the product arithmetic) and the
   workspace must be the same, untouched in between. */
taser_status_t taser_run_prep(const taser_desc_t* desc, const void* H, const void* y,
                              const void* s0, const float* tau_in, int32_t* status, void* ws,
                              size_t ws_bytes, void* stream);
taser_status_t taser_run_solve(const taser_desc_t* desc, int8_t* sbar, float* margin,
                               int32_t* status, float* L_out, void* ws, size_t ws_bytes,
                               void* stream);

/* The step size tau = alpha / ||T~||_2 (Section III-B) of every vector, as
   taser_run_prep left it in `ws` (or the tau_in it was given), copied to
   tau: float32 [V], device memory owned by the caller.  With the computed
   tau a caller can rerun the same batch with TASER_TAU_GIVEN.  Same
   descriptor and workspace rules as taser_run_solve; errors:
   TASER_ERR_ARG (tau NULL), TASER_ERR_WORKSPACE, TASER_ERR_UNSUPPORTED. */
taser_status_t taser_run_tau(const taser_desc_t* desc, const void* ws, size_t ws_bytes,
                             float* tau, void* stream);

/* ---- Calibration ------------------------------------------------------

   Measured device rates for roofline statements (no part of the detector).
   taser_calibrate launches one kernel on `stream` that keeps every SIMD busy
   with one instruction type: kind 0 float32 FMA on the vector ALUs, kind 1
   v_mfma_f32_16x16x16_bf16, kind 2 v_mfma_f32_16x16x4_f32, `iters` loop trips
   (1 .. 2^16).  out: device float32 [taser_calibrate_elements()], owned by
   the caller, overwritten with values that depend on the work.  *flops
   (host) receives the floating-point operations the launch performs; the
   caller times it.  Errors: TASER_ERR_ARG (kind, iters, NULL pointers),
   TASER_ERR_DEVICE. */
taser_status_t taser_calibrate(int32_t kind, int32_t iters, float* out, double* flops,
                               void* stream);
int32_t taser_calibrate_elements(void);

/* ---- Mixed-size batches ------------------------------------------------

   Coherent detection of V vectors of different sizes in one call: vector v
   has B_v receive antennas, U_v users and modulation mod_v, its own channel
   (complex64 B_v x U_v row-major, starting H_off[v] complex elements into H)
   and receive vector (B_v complex64 at y + y_off[v]).  The call sorts the
   vectors into size buckets on the device (N-1 <= 16, <= 32, <= 64) and runs
   one kernel per bucket; it allocates nothing, synchronises
   nothing and launches a fixed sequence of kernels (capturable into a HIP
   graph).  desc->num_vectors, prec, tau_mode, t_max, flags and alpha apply to
   every vector; desc->mode must be TASER_COHERENT; desc->B, U, mod and
   y_per_H are not used.  Outputs: sbar int8 [V][stride] and margin float32
   [V][stride] (or NULL): the first N_v - 1 entries of row v are the
   decisions / margins, the rest of the row is 0; status [V].  Vectors with U_v > 32 or N_v - 1 > 64 get status
   TASER_VEC_UNSUPPORTED.  All per-vector arrays are device arrays. */
/* Launch choices (NULL = all 0, the defaults), results do not depend on them:
     blocks[b]  grid of size bucket b: 0 launches one workgroup per vector of
                the batch, those past the bucket's count exit at once; n > 0
                (at most 2^20) a persistent grid of n workgroups that walk
                the bucket's list;
     waves[b]   register budget of bucket b's one-workgroup-per-vector
                kernel: 0 the default build, 1 the alternative (8 waves per
                SIMD for N-1 <= 16, 4 for <= 32, 3 for <= 64);
     single_launch  1: every bucket in one launch over one work queue (the
                bucket lists, largest problems first), with the registers of
                the largest size; blocks, waves and concurrent are then
                ignored;
     concurrent 1: the bucket kernels go to three streams, the caller's and
                two side streams of the library (created on the first such
                call on a device, default priority, kept until the process
                ends), forked from and joined back into the caller's stream
                with events, so that they can share the GPU; the call is
                still ordered on the caller's stream and capturable, but the
                first concurrent call on a device must not be made while a
                stream is being captured (it creates the side streams).
                Calls from several host threads are serialised while they
                enqueue. */
typedef struct {
  int32_t blocks[3];
  int32_t waves[3];
  int32_t single_launch;
  int32_t concurrent;
} taser_mixed_launch_t;

taser_status_t taser_mixed_workspace_size(const taser_desc_t* desc, size_t* bytes);

taser_status_t taser_run_mixed(const taser_desc_t* desc, const int32_t* B, const int32_t* U,
                               const int32_t* mod, const int64_t* H_off, const int64_t* y_off,
                               const void* H, const void* y, const float* tau_in, int8_t* sbar,
                               float* margin, int32_t stride, int32_t* status,
                               const taser_mixed_launch_t* launch, void* ws, size_t ws_bytes,
                               void* stream);

/* ---- Unfolded TASER (learned step sizes) --------------------------------

   Algorithm 1 with one step size per iteration, tau_t = alpha_t / lam[v],
   t = 0..t_max-1 (a constant alpha_t is the paper's algorithm), and the
   gradient of a loss with respect to alpha.  Inputs per vector: T~ [V][N][N],
   D [V][N] and lam [V] = ||T~||_2 (e.g. from taser_build_T).  real selects
   float (TASER_REAL_F32, training) or double (TASER_REAL_F64, gradient
   checks).  Every array has that element type.  N <= 64. */
enum { TASER_REAL_F32 = 0, TASER_REAL_F64 = 1 };

typedef struct {
  int32_t num_vectors;  /* V, 0..TASER_MAX_VECTORS */
  int32_t N;            /* problem size, 2..64 */
  int32_t t_max;        /* iterations, 1..10000 */
  int32_t real;         /* TASER_REAL_* */
  int32_t ckpt_every;   /* c >= 1: L is stored before iterations 0, c, 2c, ... */
  int32_t flags;        /* TASER_FLAG_LITERAL_LAST or 0 */
} taser_unfolded_t;

/* Elements (not bytes) of the checkpoint buffer: V * ceil(t_max/c) * N(N+1)/2;
   bytes of the backward workspace: V * t_max * sizeof(real). */
taser_status_t taser_unfolded_sizes(const taser_unfolded_t* u, size_t* ckpt_elems,
                                    size_t* ws_bytes);

/* Forward: L_out [V][N(N+1)/2] (packed rows) after t_max iterations; the
   checkpoints L_ckpt (layout [V][ceil(t_max/c)][N(N+1)/2]) for the backward. */
taser_status_t taser_unfolded_forward(const taser_unfolded_t* u, const void* Tt, const void* D,
                                      const void* lam, const void* alpha_t, void* L_ckpt,
                                      void* L_out, void* stream);

/* Backward: given dL [V][N(N+1)/2] = dLoss/dL_out, writes
   dalpha [t_max] = dLoss/dalpha_t summed over the batch (deterministic:
   fixed-order reduction over vectors).  ws: taser_unfolded_sizes() bytes.
   An empty batch (V = 0) writes dalpha = 0 and needs only dalpha (the other
   pointers may be NULL). */
taser_status_t taser_unfolded_backward(const taser_unfolded_t* u, const void* Tt, const void* D,
                                       const void* lam, const void* alpha_t, const void* L_ckpt,
                                       const void* dL, void* dalpha, void* ws, size_t ws_bytes,
                                       void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TASER_H */
