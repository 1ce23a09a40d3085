// extern "C" entry points of libtaser.so: argument validation and dispatch.
// Every check happens on the host before any launch; see include/taser.h.
#include <math.h>
#include <stdlib.h>

#include <atomic>

#include "taser_internal.h"

using namespace taser;

namespace {

bool valid_enums(const taser_desc_t* d) {
  if (d->mod != TASER_BPSK && d->mod != TASER_QPSK) return false;
  if (d->mode != TASER_COHERENT && d->mode != TASER_JED) return false;
  if (d->prec < TASER_PREC_F32 || d->prec > TASER_PREC_FIXED14) return false;
  if (d->tau_mode != TASER_TAU_SPECTRAL && d->tau_mode != TASER_TAU_GIVEN) return false;
  if (d->flags & ~TASER_FLAG_LITERAL_LAST) return false;
  return true;
}

taser_status_t check(const taser_desc_t* d) {
  if (!d) return TASER_ERR_ARG;
  if (!valid_enums(d)) return TASER_ERR_ARG;
  if (d->t_max < 0 || d->t_max > 100000) return TASER_ERR_ARG;
  if (d->tau_mode == TASER_TAU_SPECTRAL && !(d->alpha > 0.f && d->alpha < 1.f)) return TASER_ERR_ARG;
  if (d->num_vectors < 0 || d->num_vectors > TASER_MAX_VECTORS || d->B < 1 || d->U < 1)
    return TASER_ERR_SHAPE;
  const int N = taser_problem_size(d->U, d->mod);
  if (N < 2 || N > TASER_MAX_N) return TASER_ERR_SHAPE;
  if (d->y_per_H < 1) return TASER_ERR_SHAPE;
  if (d->mode == TASER_JED && d->y_per_H != 1) return TASER_ERR_SHAPE;
  if (d->num_vectors % d->y_per_H != 0) return TASER_ERR_SHAPE;
  return TASER_OK;
}

StagedArgs staged_args(const taser_desc_t* d) {
  StagedArgs a{};
  a.V = d->num_vectors; a.B = d->B; a.U = d->U; a.N = taser_problem_size(d->U, d->mod);
  a.mod = d->mod; a.mode = d->mode; a.y_per_H = d->y_per_H; a.t_max = d->t_max;
  a.flags = d->flags; a.tau_mode = d->tau_mode; a.alpha = d->alpha;
  return a;
}


// Host-side fault injection (taser_debug_inject_device_error): the number of
// upcoming launching calls that fail with TASER_ERR_DEVICE before they launch.
std::atomic<int> g_inject{0};

bool injected_device_error() {
  int n = g_inject.load(std::memory_order_relaxed);
  while (n > 0)
    if (g_inject.compare_exchange_weak(n, n - 1, std::memory_order_relaxed)) return true;
  return false;
}

// Every entry point that launches device work ends here: an injected fault,
// or a failed launch (the launchers return hipGetLastError()), is
// TASER_ERR_DEVICE.
template <typename F>
taser_status_t launch_status(F&& launch) {
  if (injected_device_error()) return TASER_ERR_DEVICE;
  return launch() == hipSuccess ? TASER_OK : TASER_ERR_DEVICE;
}

}  // namespace

extern "C" {

int taser_abi_version(void) { return TASER_ABI_VERSION; }

taser_status_t taser_debug_inject_device_error(int32_t count) {
  if (count < 0) return TASER_ERR_ARG;
  g_inject.store(count, std::memory_order_relaxed);
  return TASER_OK;
}

const char* taser_status_string(int status) {
  switch (status) {
    case TASER_OK: return "TASER_OK";
    case TASER_ERR_ARG: return "TASER_ERR_ARG: invalid argument (null pointer, enum, alpha or t_max)";
    case TASER_ERR_SHAPE: return "TASER_ERR_SHAPE: sizes out of range or inconsistent";
    case TASER_ERR_UNSUPPORTED: return "TASER_ERR_UNSUPPORTED: request not implemented for this shape or precision";
    case TASER_ERR_WORKSPACE: return "TASER_ERR_WORKSPACE: workspace missing or too small";
    case TASER_ERR_DEVICE: return "TASER_ERR_DEVICE: a HIP call or kernel launch failed";
    default: return "TASER: unknown status";
  }
}

int taser_problem_size(int U, int mod) {
  if (U < 1) return -1;
  if (mod == TASER_QPSK) return 2 * U + 1;
  if (mod == TASER_BPSK) return U + 1;
  return -1;
}

taser_status_t taser_check_desc(const taser_desc_t* desc) { return check(desc); }

taser_status_t taser_build_T(const taser_desc_t* desc, const void* H, const void* y,
                             const void* s0, float* Tt, float* D, float* lam, float* tau,
                             int32_t* status, void* stream) {
  taser_status_t st = check(desc);
  if (st != TASER_OK) return st;
  StagedArgs a = staged_args(desc);
  if (a.V == 0) return TASER_OK;
  const bool jed = desc->mode == TASER_JED;
  if (!y || !Tt || !D || !lam || !tau || !status) return TASER_ERR_ARG;
  if (!jed && !H) return TASER_ERR_ARG;
  if (jed && !s0) return TASER_ERR_ARG;
  const bool vec = build_T_vec_tiles(a) > 0;
  if (!vec && build_T_lds_bytes(a.B, a.U, a.N) == 0) return TASER_ERR_UNSUPPORTED;
  a.H = static_cast<const float2*>(H);
  a.y = static_cast<const float2*>(y);
  a.s0 = static_cast<const float2*>(s0);
  a.Tt = Tt; a.D = D; a.lam = lam; a.tau = tau; a.status = status;
  return launch_status([&] {
    const hipStream_t s = static_cast<hipStream_t>(stream);
    return vec ? launch_build_T_vec(a, s) : launch_build_T(a, s);
  });
}

static FixedArgs fixed_args(const taser_desc_t* d) {
  FixedArgs f{};
  f.V = d->num_vectors; f.N = taser_problem_size(d->U, d->mod); f.t_max = d->t_max;
  return f;
}

taser_status_t taser_solve(const taser_desc_t* desc, const float* Tt, const float* D,
                           const float* tau, float* L, int32_t* status, void* stream) {
  taser_status_t st = check(desc);
  if (st != TASER_OK) return st;
  if (desc->prec != TASER_PREC_F32 && desc->prec != TASER_PREC_FIXED14) return TASER_ERR_UNSUPPORTED;
  if (desc->prec == TASER_PREC_FIXED14 && taser_problem_size(desc->U, desc->mod) > 64)
    return TASER_ERR_UNSUPPORTED;
  StagedArgs a = staged_args(desc);
  if (a.V == 0) return TASER_OK;
  if (!Tt || !D || !tau || !L || !status) return TASER_ERR_ARG;
  if (desc->prec == TASER_PREC_FIXED14) {
    FixedArgs f = fixed_args(desc);
    f.Tt = Tt; f.Df = D; f.tau = tau; f.Lf = L; f.status = status;
    return launch_status([&] { return launch_fixed_solve(f, static_cast<hipStream_t>(stream)); });
  }
  return launch_status([&] {
    return launch_solve(a, Tt, D, tau, L, status, static_cast<hipStream_t>(stream));
  });
}

taser_status_t taser_detect(const taser_desc_t* desc, const float* L, const float* D,
                            int8_t* sbar, float* margin, void* stream) {
  taser_status_t st = check(desc);
  if (st != TASER_OK) return st;
  const int N = taser_problem_size(desc->U, desc->mod);
  if (desc->num_vectors == 0) return TASER_OK;
  if (!L || !D || !sbar) return TASER_ERR_ARG;
  return launch_status([&] {
    return launch_detect(desc->num_vectors, N, L, D, sbar, margin,
                         static_cast<hipStream_t>(stream));
  });
}

taser_status_t taser_fixed_quantize(const taser_desc_t* desc, const float* Tt, const float* D,
                                    const float* tau, int16_t* That, int16_t* Dq, void* stream) {
  taser_status_t st = check(desc);
  if (st != TASER_OK) return st;
  if (taser_problem_size(desc->U, desc->mod) > 64) return TASER_ERR_UNSUPPORTED;
  if (desc->num_vectors == 0) return TASER_OK;
  if (!Tt || !D || !tau || !That || !Dq) return TASER_ERR_ARG;
  const FixedArgs f = fixed_args(desc);
  return launch_status([&] {
    return launch_fixed_quantize(f, Tt, D, tau, That, Dq, static_cast<hipStream_t>(stream));
  });
}

taser_status_t taser_fixed_solve(const taser_desc_t* desc, const int16_t* That, const int16_t* Dq,
                                 int16_t* L, int8_t* sbar, int32_t* status, void* stream) {
  taser_status_t st = check(desc);
  if (st != TASER_OK) return st;
  if (taser_problem_size(desc->U, desc->mod) > 64) return TASER_ERR_UNSUPPORTED;
  if (desc->num_vectors == 0) return TASER_OK;
  if (!That || !Dq || !L || !status) return TASER_ERR_ARG;
  FixedArgs f = fixed_args(desc);
  f.That = That; f.D = Dq; f.L = L; f.sbar = sbar; f.status = status;
  return launch_status([&] { return launch_fixed_solve(f, static_cast<hipStream_t>(stream)); });
}

taser_status_t taser_reference_detect(const taser_desc_t* desc, int32_t kind, int32_t K, float n0,
                                      const void* H, const void* y, int8_t* sbar, float* soft,
                                      void* stream) {
  taser_status_t st = check(desc);
  if (st != TASER_OK) return st;
  if (kind < TASER_REF_MF || kind > TASER_REF_KBEST) return TASER_ERR_ARG;
  if (kind == TASER_REF_KBEST && (K < 1 || K > 16)) return TASER_ERR_ARG;
  if (kind == TASER_REF_MMSE && !(n0 >= 0.f && isfinite(n0))) return TASER_ERR_ARG;
  if (desc->mode != TASER_COHERENT) return TASER_ERR_UNSUPPORTED;
  const int M = taser_problem_size(desc->U, desc->mod) - 1;
  if (M > 64 || (kind == TASER_REF_ML && M > 20)) return TASER_ERR_UNSUPPORTED;
  if (desc->num_vectors == 0) return TASER_OK;
  if (!H || !y || !sbar) return TASER_ERR_ARG;
  RefArgs r{};
  r.V = desc->num_vectors; r.B = desc->B; r.U = desc->U; r.M = M; r.mod = desc->mod;
  r.y_per_H = desc->y_per_H; r.kind = kind; r.K = K; r.n0 = n0;
  r.H = static_cast<const float2*>(H);
  r.y = static_cast<const float2*>(y);
  r.sbar = sbar; r.soft = soft;
  return launch_status([&] { return launch_reference(r, static_cast<hipStream_t>(stream)); });
}

taser_status_t taser_sdr_detect(const taser_desc_t* desc, const float* Tt, const float* D,
                                const int32_t* status, int8_t* sbar, double* objective, double* gap,
                                double* X, int32_t* iterations, void* stream) {
  taser_status_t st = check(desc);
  if (st != TASER_OK) return st;
  const int N = taser_problem_size(desc->U, desc->mod);
  if (N > 65) return TASER_ERR_UNSUPPORTED;
  if (desc->num_vectors == 0) return TASER_OK;
  if (!Tt || !sbar) return TASER_ERR_ARG;
  SdrArgs r{};
  r.V = desc->num_vectors; r.N = N; r.Tt = Tt; r.D = D; r.status = status; r.sbar = sbar;
  r.objective = objective; r.gap = gap; r.X = X; r.iterations = iterations;
  return launch_status([&] { return launch_sdr(r, static_cast<hipStream_t>(stream)); });
}

taser_status_t taser_jed_channel(const taser_desc_t* desc, const void* Y, const void* s0,
                                 const int8_t* sbar, void* h, void* stream) {
  taser_status_t st = check(desc);
  if (st != TASER_OK) return st;
  if (desc->mode != TASER_JED) return TASER_ERR_ARG;
  if (desc->num_vectors == 0) return TASER_OK;
  if (!Y || !s0 || !sbar || !h) return TASER_ERR_ARG;
  return launch_status([&] {
    return launch_jed_channel(desc->num_vectors, desc->B, desc->U, desc->mod == TASER_QPSK, Y, s0,
                              sbar, h, static_cast<hipStream_t>(stream));
  });
}

static taser_status_t fused_args(const taser_desc_t* desc, FusedArgs* a) {
  taser_status_t st = check(desc);
  if (st != TASER_OK) return st;
  *a = FusedArgs{};
  a->V = desc->num_vectors; a->B = desc->B; a->U = desc->U;
  a->N = taser_problem_size(desc->U, desc->mod);
  a->mod = desc->mod; a->mode = desc->mode; a->y_per_H = desc->y_per_H; a->t_max = desc->t_max;
  a->flags = desc->flags; a->tau_mode = desc->tau_mode; a->prec = desc->prec; a->alpha = desc->alpha;
  if (desc->prec == TASER_PREC_FIXED14 || !fused_supported(*a)) return TASER_ERR_UNSUPPORTED;
  return TASER_OK;
}

taser_status_t taser_workspace_size(const taser_desc_t* desc, size_t* bytes) {
  if (!bytes) return TASER_ERR_ARG;
  FusedArgs a;
  taser_status_t st = fused_args(desc, &a);
  if (st != TASER_OK) return st;
  *bytes = fused_workspace_bytes(a);
  return TASER_OK;
}

// Argument checks and argument block of taser_run and taser_run_static
// (everything but the workspace).
static taser_status_t run_args(const taser_desc_t* desc, const void* H, const void* y,
                               const void* s0, const float* tau_in, int8_t* sbar, float* margin,
                               int32_t* status, float* L_out, FusedArgs* a) {
  taser_status_t st = fused_args(desc, a);
  if (st != TASER_OK || a->V == 0) return st;
  const bool jed = desc->mode == TASER_JED;
  if (!y || !sbar || !status) return TASER_ERR_ARG;
  if (!jed && !H) return TASER_ERR_ARG;
  if (jed && !s0) return TASER_ERR_ARG;
  if (desc->tau_mode == TASER_TAU_GIVEN && !tau_in) return TASER_ERR_ARG;
  a->H = static_cast<const float2*>(H);
  a->y = static_cast<const float2*>(y);
  a->s0 = static_cast<const float2*>(s0);
  a->tau_in = tau_in; a->sbar = sbar; a->margin = margin; a->status = status; a->L_out = L_out;
  return TASER_OK;
}

taser_status_t taser_run(const taser_desc_t* desc, const void* H, const void* y, const void* s0,
                         const float* tau_in, int8_t* sbar, float* margin, int32_t* status,
                         float* L_out, void* ws, size_t ws_bytes, void* stream) {
  FusedArgs a;
  taser_status_t st = run_args(desc, H, y, s0, tau_in, sbar, margin, status, L_out, &a);
  if (st != TASER_OK || a.V == 0) return st;
  const size_t need = fused_workspace_bytes(a);
  if (need > 0 && (!ws || ws_bytes < need)) return TASER_ERR_WORKSPACE;
  a.ws = static_cast<float*>(ws);
  return launch_status([&] { return launch_fused(a, static_cast<hipStream_t>(stream)); });
}

taser_status_t taser_run_static(const taser_desc_t* desc, const void* H, const void* y,
                                const void* s0, const float* tau_in, int8_t* sbar, float* margin,
                                int32_t* status, float* L_out, void* stream) {
  FusedArgs a;
  taser_status_t st = run_args(desc, H, y, s0, tau_in, sbar, margin, status, L_out, &a);
  if (st != TASER_OK || a.V == 0) return st;
  const size_t need = fused_workspace_bytes(a);
  if (need > static_scratch_bytes()) return TASER_ERR_WORKSPACE;
  return launch_status([&] {
    if (need > 0) {
      void* p = nullptr;
      const hipError_t e = static_scratch(&p);
      if (e != hipSuccess) return e;
      a.ws = static_cast<float*>(p);
    }
    return launch_fused(a, static_cast<hipStream_t>(stream));
  });
}

taser_status_t taser_run_prep(const taser_desc_t* desc, const void* H, const void* y,
                              const void* s0, const float* tau_in, int32_t* status, void* ws,
                              size_t ws_bytes, void* stream) {
  FusedArgs a;
  taser_status_t st = fused_args(desc, &a);
  if (st != TASER_OK) return st;
  if (!fused_group_supported(a)) return TASER_ERR_UNSUPPORTED;
  if (a.V == 0) return TASER_OK;
  const bool jed = desc->mode == TASER_JED;
  if (!y || !status) return TASER_ERR_ARG;
  if (!jed && !H) return TASER_ERR_ARG;
  if (jed && !s0) return TASER_ERR_ARG;
  if (desc->tau_mode == TASER_TAU_GIVEN && !tau_in) return TASER_ERR_ARG;
  const size_t need = fused_workspace_bytes(a);
  if (need > 0 && (!ws || ws_bytes < need)) return TASER_ERR_WORKSPACE;
  a.H = static_cast<const float2*>(H);
  a.y = static_cast<const float2*>(y);
  a.s0 = static_cast<const float2*>(s0);
  a.tau_in = tau_in; a.status = status;
  a.ws = static_cast<float*>(ws);
  return launch_status([&] { return launch_fused_prep(a, static_cast<hipStream_t>(stream)); });
}

taser_status_t taser_run_solve(const taser_desc_t* desc, int8_t* sbar, float* margin,
                               int32_t* status, float* L_out, void* ws, size_t ws_bytes,
                               void* stream) {
  FusedArgs a;
  taser_status_t st = fused_args(desc, &a);
  if (st != TASER_OK) return st;
  if (!fused_group_supported(a)) return TASER_ERR_UNSUPPORTED;
  if (a.V == 0) return TASER_OK;
  if (!sbar || !status) return TASER_ERR_ARG;
  const size_t need = fused_workspace_bytes(a);
  if (need > 0 && (!ws || ws_bytes < need)) return TASER_ERR_WORKSPACE;
  a.sbar = sbar; a.margin = margin; a.status = status; a.L_out = L_out;
  a.ws = static_cast<float*>(ws);
  return launch_status([&] { return launch_fused_solve(a, static_cast<hipStream_t>(stream)); });
}

taser_status_t taser_run_tau(const taser_desc_t* desc, const void* ws, size_t ws_bytes,
                             float* tau, void* stream) {
  FusedArgs a;
  taser_status_t st = fused_args(desc, &a);
  if (st != TASER_OK) return st;
  if (!fused_group_supported(a)) return TASER_ERR_UNSUPPORTED;
  if (a.V == 0) return TASER_OK;
  if (!tau) return TASER_ERR_ARG;
  const size_t need = fused_workspace_bytes(a);
  if (!ws || ws_bytes < need) return TASER_ERR_WORKSPACE;
  a.ws = static_cast<float*>(const_cast<void*>(ws));
  return launch_status([&] { return launch_fused_tau(a, tau, static_cast<hipStream_t>(stream)); });
}

taser_status_t taser_calibrate(int32_t kind, int32_t iters, float* out, double* flops,
                               void* stream) {
  if (kind < 0 || kind > 2 || iters < 1 || iters > (1 << 16) || !out || !flops)
    return TASER_ERR_ARG;
  return launch_status([&] {
    return launch_calibrate(kind, iters, out, flops, static_cast<hipStream_t>(stream));
  });
}

int32_t taser_calibrate_elements(void) { return calib_elements(); }

static taser_status_t mixed_check(const taser_desc_t* d) {
  if (!d) return TASER_ERR_ARG;
  if (d->prec < TASER_PREC_F32 || d->prec > TASER_PREC_FIXED14) return TASER_ERR_ARG;
  if (d->tau_mode != TASER_TAU_SPECTRAL && d->tau_mode != TASER_TAU_GIVEN) return TASER_ERR_ARG;
  if (d->flags & ~TASER_FLAG_LITERAL_LAST) return TASER_ERR_ARG;
  if (d->t_max < 0 || d->t_max > 100000) return TASER_ERR_ARG;
  if (d->tau_mode == TASER_TAU_SPECTRAL && !(d->alpha > 0.f && d->alpha < 1.f)) return TASER_ERR_ARG;
  if (d->mode != TASER_COHERENT || d->prec == TASER_PREC_FIXED14) return TASER_ERR_UNSUPPORTED;
  if (d->num_vectors < 0 || d->num_vectors > TASER_MAX_VECTORS) return TASER_ERR_SHAPE;
  return TASER_OK;
}

taser_status_t taser_mixed_workspace_size(const taser_desc_t* desc, size_t* bytes) {
  if (!bytes) return TASER_ERR_ARG;
  taser_status_t st = mixed_check(desc);
  if (st != TASER_OK) return st;
  *bytes = mixed_workspace_bytes(desc->num_vectors);
  return TASER_OK;
}

taser_status_t taser_run_mixed(const taser_desc_t* desc, const int32_t* Bv, const int32_t* Uv,
                               const int32_t* modv, const int64_t* H_off, const int64_t* y_off,
                               const void* H, const void* y, const float* tau_in, int8_t* sbar,
                               float* margin, int32_t stride, int32_t* status,
                               const taser_mixed_launch_t* launch, void* ws, size_t ws_bytes,
                               void* stream) {
  taser_status_t st = mixed_check(desc);
  if (st != TASER_OK) return st;
  if (desc->num_vectors == 0) return TASER_OK;
  if (!Bv || !Uv || !modv || !H_off || !y_off || !H || !y || !sbar || !status) return TASER_ERR_ARG;
  if (desc->tau_mode == TASER_TAU_GIVEN && !tau_in) return TASER_ERR_ARG;
  if (stride < 64) return TASER_ERR_SHAPE;
  if (launch) {
    for (int b = 0; b < kMixedBuckets; ++b) {
      if (launch->blocks[b] < 0 || launch->blocks[b] > (1 << 20)) return TASER_ERR_ARG;
      if (launch->waves[b] != 0 && launch->waves[b] != 1) return TASER_ERR_ARG;
    }
    if (launch->single_launch != 0 && launch->single_launch != 1) return TASER_ERR_ARG;
    if (launch->concurrent != 0 && launch->concurrent != 1) return TASER_ERR_ARG;
  }
  const size_t need = mixed_workspace_bytes(desc->num_vectors);
  if (!ws || ws_bytes < need) return TASER_ERR_WORKSPACE;
  FusedArgs a{};
  a.V = desc->num_vectors; a.mode = TASER_COHERENT; a.y_per_H = 1; a.t_max = desc->t_max;
  a.flags = desc->flags; a.tau_mode = desc->tau_mode; a.prec = desc->prec; a.alpha = desc->alpha;
  a.H = static_cast<const float2*>(H);
  a.y = static_cast<const float2*>(y);
  a.tau_in = tau_in; a.sbar = sbar; a.margin = margin; a.status = status;
  MixedArgs m{};
  m.Bv = Bv; m.Uv = Uv; m.modv = modv; m.H_off = H_off; m.y_off = y_off; m.stride = stride;
  m.count = static_cast<int32_t*>(ws);
  m.list = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + 256);
  return launch_status([&] {
    return launch_mixed(a, m, launch, static_cast<hipStream_t>(stream));
  });
}

static taser_status_t unf_check(const taser_unfolded_t* u) {
  if (!u) return TASER_ERR_ARG;
  if (u->real != TASER_REAL_F32 && u->real != TASER_REAL_F64) return TASER_ERR_ARG;
  if (u->flags & ~TASER_FLAG_LITERAL_LAST) return TASER_ERR_ARG;
  if (u->num_vectors < 0 || u->num_vectors > TASER_MAX_VECTORS || u->N < 2 || u->N > 64)
    return TASER_ERR_SHAPE;
  if (u->t_max < 1 || u->t_max > 10000 || u->ckpt_every < 1) return TASER_ERR_SHAPE;
  UnfoldedArgs a{u->num_vectors, u->N, u->t_max, u->real, u->ckpt_every, u->flags};
  if (unfolded_lds_bytes(a) > 163840) return TASER_ERR_UNSUPPORTED;
  return TASER_OK;
}

taser_status_t taser_unfolded_sizes(const taser_unfolded_t* u, size_t* ckpt_elems,
                                    size_t* ws_bytes) {
  taser_status_t st = unf_check(u);
  if (st != TASER_OK) return st;
  if (!ckpt_elems || !ws_bytes) return TASER_ERR_ARG;
  const size_t P = (size_t)u->N * (u->N + 1) / 2;
  const size_t nck = (size_t)(u->t_max + u->ckpt_every - 1) / u->ckpt_every;
  *ckpt_elems = (size_t)u->num_vectors * nck * P;
  UnfoldedArgs a{u->num_vectors, u->N, u->t_max, u->real, u->ckpt_every, u->flags};
  *ws_bytes = unfolded_workspace_bytes(a);
  return TASER_OK;
}

taser_status_t taser_unfolded_forward(const taser_unfolded_t* u, const void* Tt, const void* D,
                                      const void* lam, const void* alpha_t, void* L_ckpt,
                                      void* L_out, void* stream) {
  taser_status_t st = unf_check(u);
  if (st != TASER_OK) return st;
  if (u->num_vectors == 0) return TASER_OK;
  if (!Tt || !D || !lam || !alpha_t || !L_ckpt || !L_out) return TASER_ERR_ARG;
  UnfoldedArgs a{u->num_vectors, u->N, u->t_max, u->real, u->ckpt_every, u->flags};
  return launch_status([&] {
    return launch_unfolded_forward(a, Tt, D, lam, alpha_t, L_ckpt, L_out,
                                   static_cast<hipStream_t>(stream));
  });
}

taser_status_t taser_unfolded_backward(const taser_unfolded_t* u, const void* Tt, const void* D,
                                       const void* lam, const void* alpha_t, const void* L_ckpt,
                                       const void* dL, void* dalpha, void* ws, size_t ws_bytes,
                                       void* stream) {
  taser_status_t st = unf_check(u);
  if (st != TASER_OK) return st;
  if (!dalpha) return TASER_ERR_ARG;
  if (u->num_vectors > 0 && (!Tt || !D || !lam || !alpha_t || !L_ckpt || !dL)) return TASER_ERR_ARG;
  UnfoldedArgs a{u->num_vectors, u->N, u->t_max, u->real, u->ckpt_every, u->flags};
  const size_t need = unfolded_workspace_bytes(a);
  if (need > 0 && (!ws || ws_bytes < need)) return TASER_ERR_WORKSPACE;
  // an empty batch still writes dalpha (zeros: the sum over no vectors)
  return launch_status([&] {
    return launch_unfolded_backward(a, Tt, D, lam, alpha_t, L_ckpt, dL, dalpha, ws,
                                    static_cast<hipStream_t>(stream));
  });
}

}  // extern "C"
