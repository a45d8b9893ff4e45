// Host implementation of the C ABI in include/lbm.h: argument validation,
// device allocation, stream binding, dispatch of the kernels and error
// reporting.  No function throws or aborts across the ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"

using Ctx = lbm_ctx;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_OR_FAIL(expr, what)             \
  do {                                      \
    hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

size_t word_of(int precision) { return precision == LBM_FP64 ? sizeof(double) : sizeof(float); }

int select_device(Ctx* c) {
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != c->device) HIP_OR_FAIL(hipSetDevice(c->device), "hipSetDevice");
  return LBM_OK;
}

int ensure_scratch(Ctx* c) {
  if (!c->fields) {
    HIP_OR_FAIL(hipMalloc(&c->fields, sizeof(double) * 6 * (size_t)c->N), "hipMalloc(fields)");
  }
  if (!c->partial) {
    c->partial_blocks = lbm::diag_blocks(*c);
    HIP_OR_FAIL(hipMalloc(&c->partial, sizeof(double) * lbm::kNumDiag * (size_t)c->partial_blocks),
                "hipMalloc(partial)");
    HIP_OR_FAIL(hipMalloc(&c->diag_dev, sizeof(double) * lbm::kNumDiag), "hipMalloc(diag)");
  }
  return LBM_OK;
}

void fill_params(Ctx* c) {
  lbm::StepParams& p = c->sp;
  const int D = c->lattice;
  p.nx = (int)c->n[0];
  p.ny = (int)c->n[1];
  p.nz = (int)c->n[2];
  for (int a = 0; a < 3; ++a) p.bc[a] = c->opt.bc[a];
  p.ps = c->ps;
  p.ms = c->ms;
  p.plane = (int)(D == 3 ? c->n[0] * c->n[1] : c->n[0]);
  const int nm = (D == 3) ? p.nz : p.ny;
  p.tiles_x = (p.nx + c->tile.bx - 1) / c->tile.bx;
  p.tiles_y = (D == 3) ? (p.ny + c->tile.by - 1) / c->tile.by : 1;
  p.chunk_len = c->tile.chunk;
  p.chunks = (nm + p.chunk_len - 1) / p.chunk_len;
  p.nblocks = p.tiles_x * p.tiles_y * p.chunks;
  p.deriv = c->opt.deriv_scheme;
  p.Cv = 1.0 / (c->gamma - 1.0);
  p.inv_Cv = c->gamma - 1.0;
  p.Pr = c->Pr;
  p.gamma = c->gamma;
  p.mu0 = c->mu;
  p.visc_exp = c->opt.visc_exponent;
  p.inv_Tref = 1.0 / c->opt.T_ref;
  if (c->precision == LBM_FP32_DEV) {
    // The rest state is taken at FP32-representable values: the kernels build
    // the rest factors in FP32 and the deviations of rho and T in FP64, and
    // both must refer to the same (rho0, T0) for exact conservation.
    // C_v likewise: g^eq is built with the FP32 C_v and T is recovered with
    // its exact FP64 inverse.
    p.Cv = (double)(float)p.Cv;
    p.inv_Cv = 1.0 / p.Cv;
    p.rho0 = (double)(float)c->opt.rho_ref;
    p.T0 = (double)(float)c->opt.T_ref;
    double u2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double u0 = a < D ? (double)(float)c->opt.u_ref[a] : 0.0;
      p.u0[a] = u0;
      p.j0[a] = p.rho0 * u0;
      u2 += u0 * u0;
      // product-form factors of the reference populations along axis a:
      // f-factors Psi_c(u0, P0) (equal to the a-factors of g^eq) and the
      // b-factors of g^eq at (u0, T0)
      const double P0 = p.T0 + u0 * u0;
      const double B1 = 0.5 * u0 * (u0 * u0 + 2.0 * p.T0);
      const double B2 = 0.5 * (u0 * u0 * u0 * u0 + 5.0 * u0 * u0 * p.T0 + 2.0 * p.T0 * p.T0);
      p.P0[a] = P0;
      p.psi0[a][0] = 0.5 * (-u0 + P0);
      p.psi0[a][1] = 1.0 - P0;
      p.psi0[a][2] = 0.5 * (u0 + P0);
      p.b0[a][0] = 0.5 * (-B1 + B2);
      p.b0[a][1] = 0.5 * u0 * u0 - B2;
      p.b0[a][2] = 0.5 * (B1 + B2);
    }
    p.rhoE0 = p.rho0 * (p.Cv * p.T0 + 0.5 * u2);  // sum_i g_i of the reference
  } else {
    p.rho0 = p.T0 = p.rhoE0 = 0.0;
    for (int a = 0; a < 3; ++a) {
      p.u0[a] = p.j0[a] = p.P0[a] = 0.0;
      for (int c = 0; c < 3; ++c) p.psi0[a][c] = p.b0[a][c] = 0.0;
    }
  }
  for (int a = 0; a < 3; ++a) {
    p.u0f[a] = (float)p.u0[a];
    p.P0f[a] = (float)p.P0[a];
    for (int c = 0; c < 3; ++c) {
      p.psi0f[a][c] = (float)p.psi0[a][c];
      p.b0f[a][c] = (float)p.b0[a][c];
    }
  }
}

bool fields_valid_host(const double* rho, const double* u, const double* T, int64_t N, int D) {
  for (int64_t n = 0; n < N; ++n) {
    if (!std::isfinite(rho[n]) || !std::isfinite(T[n]) || !(rho[n] > 0.0) || !(T[n] > 0.0)) return false;
    for (int a = 0; a < D; ++a)
      if (!std::isfinite(u[a * N + n])) return false;
  }
  return true;
}

}  // namespace

extern "C" {

void lbm_default_options(lbm_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof *opt);
  opt->precision = LBM_FP64;
  opt->bc[0] = opt->bc[1] = opt->bc[2] = LBM_BC_PERIODIC;
  opt->visc_exponent = 0.0;
  opt->T_ref = 1.0 / 3.0;
  opt->rho_ref = 1.0;
  opt->deriv_scheme = LBM_DERIV_UPWIND;
}

const char* lbm_last_error(lbm_handle) { return g_err.c_str(); }

int lbm_create(lbm_handle* out, int lattice, const int64_t dims[3], double gamma, double Pr, double mu,
               const lbm_options* opt_in) {
  if (!out) return fail(LBM_EINVAL, "lbm_create: out is NULL");
  *out = nullptr;
  if (lattice != LBM_D2Q9 && lattice != LBM_D3Q27) return fail(LBM_EINVAL, "lbm_create: lattice must be 2 or 3");
  if (!dims) return fail(LBM_EINVAL, "lbm_create: dims is NULL");
  for (int a = 0; a < 3; ++a)
    if (dims[a] < 1 || dims[a] > (int64_t)1 << 30) return fail(LBM_EINVAL, "lbm_create: dims out of range");
  if (lattice == LBM_D2Q9 && dims[2] != 1) return fail(LBM_EINVAL, "lbm_create: D2Q9 needs dims[2] == 1");
  if (!(gamma > 1.0) || !std::isfinite(gamma)) return fail(LBM_EINVAL, "lbm_create: gamma must be > 1");
  if (!(Pr > 0.0) || !std::isfinite(Pr)) return fail(LBM_EINVAL, "lbm_create: Pr must be > 0");
  if (!(mu > 0.0) || !std::isfinite(mu)) return fail(LBM_EINVAL, "lbm_create: mu must be > 0");
  lbm_options opt;
  lbm_default_options(&opt);
  if (opt_in) opt = *opt_in;
  if (opt.precision != LBM_FP64 && opt.precision != LBM_FP32_DEV)
    return fail(LBM_EINVAL, "lbm_create: unknown precision");
  for (int a = 0; a < 3; ++a)
    if (opt.bc[a] != LBM_BC_PERIODIC && opt.bc[a] != LBM_BC_ZERO_GRADIENT)
      return fail(LBM_EINVAL, "lbm_create: unknown boundary kind");
  if (opt.deriv_scheme != LBM_DERIV_UPWIND && opt.deriv_scheme != LBM_DERIV_CENTRAL)
    return fail(LBM_EINVAL, "lbm_create: unknown derivative scheme");
  if (!std::isfinite(opt.visc_exponent)) return fail(LBM_EINVAL, "lbm_create: bad viscosity exponent");
  if (!(opt.T_ref > 0.0) || !std::isfinite(opt.T_ref)) return fail(LBM_EINVAL, "lbm_create: T_ref must be > 0");
  if (!(opt.rho_ref > 0.0) || !std::isfinite(opt.rho_ref)) return fail(LBM_EINVAL, "lbm_create: rho_ref must be > 0");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(opt.u_ref[a]) || std::fabs(opt.u_ref[a]) >= 1.0)
      return fail(LBM_EINVAL, "lbm_create: u_ref components must be finite and |u_ref| < 1");
  const int64_t N = dims[0] * dims[1] * dims[2];
  if (N > ((int64_t)1 << 31) - 1024) return fail(LBM_EINVAL, "lbm_create: more than 2^31 nodes");

  lbm::Tile tile = lbm::default_tile(lattice, opt.precision, dims);
  if (opt.tile[0] || opt.tile[1] || opt.tile[2]) {
    lbm::Tile t{opt.tile[0] ? opt.tile[0] : tile.bx, opt.tile[1] ? opt.tile[1] : tile.by,
                opt.tile[2] ? opt.tile[2] : tile.chunk};
    if (lattice == LBM_D2Q9 && !opt.tile[1]) t.by = 1;
    if (!lbm::tile_supported(lattice, opt.precision, t) || t.chunk < 1) return fail(LBM_EINVAL, "lbm_create: launch tile not available");
    tile = t;
  }

  Ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(LBM_ENOMEM, "lbm_create: host allocation failed");
  c->lattice = lattice;
  c->Q = lattice == 2 ? 9 : 27;
  c->precision = opt.precision;
  for (int a = 0; a < 3; ++a) c->n[a] = dims[a];
  c->N = N;
  // plane-major layout: per march plane, 2Q in-plane arrays; each array is
  // 64-element aligned and the arrays are staggered by 64 elements
  {
    const int64_t plane = lattice == 3 ? dims[0] * dims[1] : dims[0];
    c->nm = (int)(lattice == 3 ? dims[2] : dims[1]);
    c->ps = ((plane + 63) / 64) * 64 + 64;
    c->ms = c->ps * 2 * c->Q;
  }
  c->gamma = gamma;
  c->Pr = Pr;
  c->mu = mu;
  c->opt = opt;
  c->tile = tile;
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipGetDevice");
  }
  fill_params(c);
  const size_t bytes = word_of(c->precision) * (size_t)c->nm * (size_t)c->ms;
  for (int k = 0; k < 2; ++k) {
    e = hipMalloc(&c->buf[k], bytes);
    if (e != hipSuccess) {
      lbm_destroy(c);
      return fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE,
                  std::string("hipMalloc(populations): ") + hipGetErrorString(e));
    }
  }
  *out = c;
  g_err.clear();
  return LBM_OK;
}

int lbm_destroy(lbm_handle h) {
  if (!h) return LBM_OK;
  Ctx* c = h;
  select_device(c);
  if (c->stream) hipStreamSynchronize(c->stream);
  for (int k = 0; k < 2; ++k)
    if (c->buf[k]) hipFree(c->buf[k]);
  if (c->fields) hipFree(c->fields);
  if (c->partial) hipFree(c->partial);
  if (c->diag_dev) hipFree(c->diag_dev);
  delete c;
  return LBM_OK;
}

int lbm_set_stream(lbm_handle h, void* stream) {
  if (!h) return fail(LBM_EINVAL, "lbm_set_stream: NULL handle");
  h->stream = static_cast<hipStream_t>(stream);
  return LBM_OK;
}

int lbm_init_fields(lbm_handle h, const double* rho, const double* u, const double* T, int mem) {
  if (!h) return fail(LBM_EINVAL, "lbm_init_fields: NULL handle");
  if (!rho || !u || !T) return fail(LBM_EINVAL, "lbm_init_fields: NULL field");
  if (mem != LBM_HOST && mem != LBM_DEVICE) return fail(LBM_EINVAL, "lbm_init_fields: bad memory kind");
  Ctx* c = h;
  int rc = select_device(c);
  if (rc) return rc;
  const int64_t N = c->N;
  const int D = c->lattice;
  if ((rc = ensure_scratch(c))) return rc;
  const double *drho = rho, *du = u, *dT = T;
  if (mem == LBM_HOST) {
    if (!fields_valid_host(rho, u, T, N, D))
      return fail(LBM_EINVAL, "lbm_init_fields: non-finite value or rho <= 0 or T <= 0");
    double* F = c->fields;
    HIP_OR_FAIL(hipMemcpyAsync(F, rho, sizeof(double) * N, hipMemcpyHostToDevice, c->stream), "copy rho");
    HIP_OR_FAIL(hipMemcpyAsync(F + N, u, sizeof(double) * N * D, hipMemcpyHostToDevice, c->stream), "copy u");
    HIP_OR_FAIL(hipMemcpyAsync(F + 4 * N, T, sizeof(double) * N, hipMemcpyHostToDevice, c->stream), "copy T");
    drho = F;
    du = F + N;
    dT = F + 4 * N;
  } else {
    HIP_OR_FAIL(lbm::launch_validate(*c, rho, u, T, c->partial, c->partial_blocks, c->diag_dev), "validate");
    double bad = 0.0;
    HIP_OR_FAIL(hipMemcpyAsync(&bad, c->diag_dev, sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy count");
    HIP_OR_FAIL(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (bad != 0.0) return fail(LBM_EINVAL, "lbm_init_fields: non-finite value or rho <= 0 or T <= 0");
  }
  HIP_OR_FAIL(lbm::launch_init(*c, drho, du, dT, c->buf[0]), "init kernel");
  if (mem == LBM_HOST) HIP_OR_FAIL(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  c->cur = 0;
  c->step = 0;
  c->initialised = true;
  c->unstable = false;
  return LBM_OK;
}

int lbm_step(lbm_handle h, int64_t n) {
  if (!h) return fail(LBM_EINVAL, "lbm_step: NULL handle");
  if (n < 0) return fail(LBM_EINVAL, "lbm_step: n < 0");
  Ctx* c = h;
  if (!c->initialised) return fail(LBM_ESTATE, "lbm_step: call lbm_init_fields first");
  if (c->unstable) return fail(LBM_EUNSTABLE, "lbm_step: the state has non-finite or non-positive rho/T");
  int rc = select_device(c);
  if (rc) return rc;
  for (int64_t k = 0; k < n; ++k) {
    HIP_OR_FAIL(lbm::launch_step(*c, c->buf[c->cur], c->buf[c->cur ^ 1]), "step kernel");
    c->cur ^= 1;
    c->step += 1;
  }
  return LBM_OK;
}

int lbm_moments(lbm_handle h, double* rho, double* u, double* T, int mem) {
  if (!h) return fail(LBM_EINVAL, "lbm_moments: NULL handle");
  if (mem != LBM_HOST && mem != LBM_DEVICE) return fail(LBM_EINVAL, "lbm_moments: bad memory kind");
  Ctx* c = h;
  if (!c->initialised) return fail(LBM_ESTATE, "lbm_moments: call lbm_init_fields first");
  int rc = select_device(c);
  if (rc) return rc;
  if ((rc = ensure_scratch(c))) return rc;
  const int64_t N = c->N;
  HIP_OR_FAIL(lbm::launch_fields(*c, c->buf[c->cur], c->fields), "moments kernel");
  const hipMemcpyKind kind = mem == LBM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  if (rho) HIP_OR_FAIL(hipMemcpyAsync(rho, c->fields, sizeof(double) * N, kind, c->stream), "copy rho");
  if (u) HIP_OR_FAIL(hipMemcpyAsync(u, c->fields + N, sizeof(double) * N * c->lattice, kind, c->stream), "copy u");
  if (T) HIP_OR_FAIL(hipMemcpyAsync(T, c->fields + 4 * N, sizeof(double) * N, kind, c->stream), "copy T");
  if (mem == LBM_HOST) HIP_OR_FAIL(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  return LBM_OK;
}

int lbm_diagnostics(lbm_handle h, lbm_diag* out) {
  if (!h || !out) return fail(LBM_EINVAL, "lbm_diagnostics: NULL argument");
  Ctx* c = h;
  if (!c->initialised) return fail(LBM_ESTATE, "lbm_diagnostics: call lbm_init_fields first");
  int rc = select_device(c);
  if (rc) return rc;
  if ((rc = ensure_scratch(c))) return rc;
  HIP_OR_FAIL(lbm::launch_fields(*c, c->buf[c->cur], c->fields), "moments kernel");
  HIP_OR_FAIL(lbm::launch_diag(*c, c->fields, c->partial, c->partial_blocks, c->diag_dev), "diagnostics kernel");
  double v[lbm::kNumDiag];
  HIP_OR_FAIL(hipMemcpyAsync(v, c->diag_dev, sizeof v, hipMemcpyDeviceToHost, c->stream), "copy diagnostics");
  HIP_OR_FAIL(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  std::memset(out, 0, sizeof *out);
  out->step = c->step;
  out->mass = v[0];
  out->momentum[0] = v[1];
  out->momentum[1] = v[2];
  out->momentum[2] = v[3];
  out->energy = v[4];
  out->kinetic_energy = v[5];
  out->dilatation_sq_sum = v[6];
  out->u2_sum = v[7];
  out->cs_sum = v[8];
  out->rho2_sum = v[9];
  out->vorticity_sq_sum = v[10];
  out->dissipation_sum = v[11];
  for (int a = 0; a < 3; ++a) {
    out->u_axis_sq_sum[a] = v[12 + a];
    out->du_axis_sq_sum[a] = v[15 + a];
  }
  out->nonfinite = (int64_t)v[18];
  out->nonpositive = (int64_t)v[19];
  out->nodes = (int64_t)v[20];
  c->unstable = out->nonfinite > 0 || out->nonpositive > 0;
  return LBM_OK;
}

size_t lbm_state_bytes(lbm_handle h) {
  if (!h) return 0;
  return word_of(h->precision) * (size_t)(2 * h->Q) * (size_t)h->N;
}

int lbm_get_state(lbm_handle h, void* buf, size_t bytes, int mem) {
  if (!h || !buf) return fail(LBM_EINVAL, "lbm_get_state: NULL argument");
  if (mem != LBM_HOST && mem != LBM_DEVICE) return fail(LBM_EINVAL, "lbm_get_state: bad memory kind");
  Ctx* c = h;
  if (!c->initialised) return fail(LBM_ESTATE, "lbm_get_state: no state yet");
  if (bytes != lbm_state_bytes(h)) return fail(LBM_EINVAL, "lbm_get_state: wrong buffer size");
  int rc = select_device(c);
  if (rc) return rc;
  // pack into the other population buffer (its content is dead between steps), then copy out
  void* scratch = c->buf[c->cur ^ 1];
  HIP_OR_FAIL(lbm::launch_pack(*c, c->buf[c->cur], scratch), "pack kernel");
  HIP_OR_FAIL(hipMemcpyAsync(buf, scratch, bytes, mem == LBM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                             c->stream),
              "copy state");
  if (mem == LBM_HOST) HIP_OR_FAIL(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  return LBM_OK;
}

int lbm_set_state(lbm_handle h, const void* buf, size_t bytes, int mem, int64_t step) {
  if (!h || !buf) return fail(LBM_EINVAL, "lbm_set_state: NULL argument");
  if (mem != LBM_HOST && mem != LBM_DEVICE) return fail(LBM_EINVAL, "lbm_set_state: bad memory kind");
  if (step < 0) return fail(LBM_EINVAL, "lbm_set_state: step < 0");
  Ctx* c = h;
  if (bytes != lbm_state_bytes(h)) return fail(LBM_EINVAL, "lbm_set_state: wrong buffer size");
  int rc = select_device(c);
  if (rc) return rc;
  HIP_OR_FAIL(hipMemcpyAsync(c->buf[1], buf, bytes, mem == LBM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                             c->stream),
              "copy state");
  HIP_OR_FAIL(lbm::launch_unpack(*c, c->buf[1], c->buf[0]), "unpack kernel");
  if (mem == LBM_HOST) HIP_OR_FAIL(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  c->cur = 0;
  c->step = step;
  c->initialised = true;
  c->unstable = false;
  return LBM_OK;
}

int64_t lbm_step_count(lbm_handle h) { return h ? h->step : -1; }

int lbm_device_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src) return fail(LBM_EINVAL, "lbm_device_copy: NULL pointer");
  if (bytes % 16) return fail(LBM_EINVAL, "lbm_device_copy: bytes must be a multiple of 16");
  if (((uintptr_t)dst | (uintptr_t)src) % 16) return fail(LBM_EINVAL, "lbm_device_copy: pointers must be 16-byte aligned");
  HIP_OR_FAIL(lbm::launch_copy(dst, src, bytes, static_cast<hipStream_t>(stream)), "copy kernel");
  return LBM_OK;
}

}  // extern "C"
