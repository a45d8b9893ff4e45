// Host implementation of the C ABI in include/lbm.h: argument validation,
// device allocation, stream binding, dispatch of the kernels and error
// reporting.  No function throws or aborts across the ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
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

}  // namespace

int lbm::set_error(int code, const std::string& msg) { return fail(code, msg); }

namespace {

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

// Step parameters of handle c for launch tile t.
void fill_step_params(const lbm::Ctx* c, const lbm::Tile& t, lbm::StepParams& p) {
  const int D = c->lattice;
  p.nx = (int)c->n[0];
  p.ny = (int)c->n[1];
  p.nz = (int)c->n[2];
  for (int a = 0; a < 3; ++a) p.bc[a] = c->opt.bc[a];
  p.sl = c->sl;
  p.blk = c->blk;
  p.ms = c->ms;
  p.plane = (int)(D == 3 ? c->n[0] * c->n[1] : c->n[0]);
  const int nm = (D == 3) ? p.nz : p.ny;
  p.tiles_x = (p.nx + t.bx - 1) / t.bx;
  p.tiles_y = (D == 3) ? (p.ny + t.by - 1) / t.by : 1;
  p.chunk_len = t.chunk;
  p.chunks = (nm + p.chunk_len - 1) / p.chunk_len;
  p.nblocks = p.tiles_x * p.tiles_y * p.chunks;
  p.deriv = c->opt.deriv_scheme;
  const double* cvp = c->opt.cv_poly;
  p.caloric = (cvp[0] != 0.0 || cvp[1] != 0.0 || cvp[2] != 0.0) ? 1 : 0;
  p.Cv = p.caloric ? cvp[0] : 1.0 / (c->gamma - 1.0);
  p.inv_Cv = p.caloric ? 1.0 / cvp[0] : c->gamma - 1.0;
  p.cv1 = p.caloric ? cvp[1] : 0.0;
  p.cv2 = p.caloric ? cvp[2] : 0.0;
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
    p.cv1 = (double)(float)p.cv1;
    p.cv2 = (double)(float)p.cv2;
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
    p.U0 = p.caloric ? lbm::caloric_u(p.Cv, p.cv1, p.cv2, p.T0) : p.Cv * p.T0;
    p.rhoE0 = p.rho0 * (p.U0 + 0.5 * u2);  // sum_i g_i of the reference
  } else {
    p.rho0 = p.T0 = p.rhoE0 = p.U0 = 0.0;
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

void fill_params(Ctx* c) { fill_step_params(c, c->tile, c->sp); }

bool fields_valid_host(const double* rho, const double* u, const double* T, int64_t N, int D) {
  for (int64_t n = 0; n < N; ++n) {
    if (!std::isfinite(rho[n]) || !std::isfinite(T[n]) || !(rho[n] > 0.0) || !(T[n] > 0.0)) return false;
    for (int a = 0; a < D; ++a)
      if (!std::isfinite(u[a * N + n])) return false;
  }
  return true;
}

// The device address of the allocation-free diagnostics' scratch array on
// each device, obtained once per device with that device current.
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
double* g_scratch[kMaxDevices] = {};

int scratch_for_device(int device, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return fail(LBM_EDEVICE, "scratch: device index beyond 63");
  if (!g_scratch[device]) {
    double* ptr = nullptr;
    const hipError_t e = lbm::scratch_address(&ptr);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch[device] = ptr;
  }
  *out = g_scratch[device];
  return LBM_OK;
}

// The 21 sums of the diagnostic reduction into the ABI struct; sets the
// handle's instability flag.
void diag_from_sums(Ctx* c, const double* v, lbm_diag* out) {
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
}

}  // namespace

// For the corrector (lbm_nn.hip): the moments of the stored state into
// c->fields (rho, u_x, u_y, u_z, T, rho E planes) on the handle's stream, and
// increments applied by re-equilibration without validation or host
// synchronisation (the caller bounds them).
int lbm::fields_current(lbm::Ctx* base) {
  lbm_ctx* c = static_cast<lbm_ctx*>(base);  // every handle is an lbm_ctx
  if (!c->initialised) return fail(LBM_ESTATE, "corrector: no state (lbm_init_fields)");
  int rc = ::select_device(c);
  if (rc) return rc;
  if ((rc = ::ensure_scratch(c))) return rc;
  HIP_OR_FAIL(lbm::launch_fields(*c, c->buf[c->cur], c->fields), "moments kernel");
  return LBM_OK;
}

int lbm::fields_increment_async(Ctx* c, const double* drho, const double* du, const double* dT) {
  if (!c->work) HIP_OR_FAIL(hipMalloc(&c->work, sizeof(double) * 10 * (size_t)c->N), "hipMalloc(work)");
  HIP_OR_FAIL(lbm::launch_fields_plus(*c, c->fields, drho, du, dT, c->work, true), "increment kernel");
  HIP_OR_FAIL(lbm::launch_fields_add(*c, c->buf[c->cur], c->fields, c->work), "re-equilibration kernel");
  return LBM_OK;
}

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
  const bool caloric = opt.cv_poly[0] != 0.0 || opt.cv_poly[1] != 0.0 || opt.cv_poly[2] != 0.0;
  if (caloric)
    if (!(opt.cv_poly[0] > 0.0 && opt.cv_poly[1] >= 0.0 && opt.cv_poly[2] >= 0.0) ||
        !std::isfinite(opt.cv_poly[0] + opt.cv_poly[1] + opt.cv_poly[2]))
      return fail(LBM_EINVAL, "lbm_create: cv_poly needs cv_poly[0] > 0 and cv_poly[1], cv_poly[2] >= 0 (finite)");
  const int64_t N = dims[0] * dims[1] * dims[2];
  if (N > ((int64_t)1 << 31) - 1024) return fail(LBM_EINVAL, "lbm_create: more than 2^31 nodes");
  // plane-major layout (see StepParams).  Slot rows: per march plane, Q slot
  // rows of (f, g) pairs, each 64-pair aligned and staggered by 64 pairs.
  // Blocks: the same formula with 64-node blocks holding their Q slots of 64
  // pairs one after the other (sl = 128, blk = 128 Q).
  if (opt.layout != LBM_LAYOUT_SLOT_ROWS && opt.layout != LBM_LAYOUT_BLOCKS)
    return fail(LBM_EINVAL, "lbm_create: unknown layout");
  const int64_t plane = lattice == 3 ? dims[0] * dims[1] : dims[0];
  const int64_t Qn = lattice == 2 ? 9 : 27;
  int64_t sl, blk, ms;
  if (opt.layout == LBM_LAYOUT_SLOT_ROWS) {
    const int64_t ps = ((plane + 63) / 64) * 64 + 64;
    sl = 2 * ps;
    blk = 128;
    ms = sl * Qn;
  } else {
    sl = 128;
    blk = 128 * Qn;
    ms = ((plane + 63) / 64) * blk;
  }
  // The step kernel addresses one march plane through a buffer resource with
  // 32-bit offsets.
  if (ms * (int64_t)word_of(opt.precision) >= ((int64_t)1 << 32))
    return fail(LBM_EINVAL, "lbm_create: one march plane of populations exceeds 4 GiB");

  lbm::Tile tile = lbm::default_tile(lattice, opt.precision, dims, caloric);
  if (opt.tile[0] || opt.tile[1] || opt.tile[2]) {
    lbm::Tile t{opt.tile[0] ? opt.tile[0] : tile.bx, opt.tile[1] ? opt.tile[1] : tile.by, opt.tile[2]};
    if (lattice == LBM_D2Q9 && !opt.tile[1]) t.by = 1;
    if (!t.chunk && t.bx > 0 && t.by > 0) t.chunk = lbm::default_chunk(lattice, dims, t.bx, t.by);
    if (!lbm::tile_supported(lattice, opt.precision, t, caloric) || t.chunk < 1)
      return fail(LBM_EINVAL, caloric ? "lbm_create: with cv_poly only the default launch shape is compiled"
                                      : "lbm_create: launch tile not available");
    tile = t;
  }

  Ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(LBM_ENOMEM, "lbm_create: host allocation failed");
  c->lattice = lattice;
  c->Q = lattice == 2 ? 9 : 27;
  c->precision = opt.precision;
  for (int a = 0; a < 3; ++a) c->n[a] = dims[a];
  c->N = N;
  c->nm = (int)(lattice == 3 ? dims[2] : dims[1]);
  c->sl = sl;
  c->blk = blk;
  c->ms = ms;
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
  {
    // set-up of the allocation-free diagnostics on this device (the entry
    // point retries and reports a failure itself)
    double* sc = nullptr;
    const std::string keep = g_err;
    if (scratch_for_device(c->device, &sc) != LBM_OK) g_err = keep;
  }
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
  // Teardown is best effort: errors here have nowhere to go.
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (int k = 0; k < 2; ++k)
    if (c->buf[k]) (void)hipFree(c->buf[k]);
  if (c->fields) (void)hipFree(c->fields);
  if (c->work) (void)hipFree(c->work);
  if (c->partial) (void)hipFree(c->partial);
  if (c->diag_dev) (void)hipFree(c->diag_dev);
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

int lbm_pattern_reference(lbm_handle h, int64_t launches) {
  if (!h) return fail(LBM_EINVAL, "lbm_pattern_reference: NULL handle");
  if (launches < 0) return fail(LBM_EINVAL, "lbm_pattern_reference: launches < 0");
  Ctx* c = h;
  if (!c->initialised) return fail(LBM_ESTATE, "lbm_pattern_reference: call lbm_init_fields first");
  if (c->sp.caloric) return fail(LBM_EINVAL, "lbm_pattern_reference: not compiled for the general caloric law");
  int rc = select_device(c);
  if (rc) return rc;
  for (int64_t k = 0; k < launches; ++k)
    HIP_OR_FAIL(lbm::launch_pattern(*c, c->buf[c->cur], c->buf[c->cur ^ 1]), "pattern kernel");
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
  diag_from_sums(c, v, out);
  return LBM_OK;
}

int lbm_diagnostics_noalloc(lbm_handle h, lbm_diag* out) {
  if (!h || !out) return fail(LBM_EINVAL, "lbm_diagnostics_noalloc: NULL argument");
  Ctx* c = h;
  if (!c->initialised) return fail(LBM_ESTATE, "lbm_diagnostics_noalloc: call lbm_init_fields first");
  int rc = select_device(c);
  if (rc) return rc;
  const int nblocks = lbm::diag_blocks(*c);
  if (nblocks < 1 || nblocks > lbm::kMaxDiagBlocks)
    return fail(LBM_EINVAL, "lbm_diagnostics_noalloc: the reduction needs more partial sums than the scratch holds");
  double* sc = nullptr;
  if ((rc = scratch_for_device(c->device, &sc))) return rc;
  double* final_sums = sc + (size_t)lbm::kMaxDiagBlocks * lbm::kNumDiag;
  HIP_OR_FAIL(lbm::launch_diag_direct(*c, c->buf[c->cur], sc, nblocks, final_sums), "diagnostics kernel");
  double v[lbm::kNumDiag];
  HIP_OR_FAIL(hipMemcpyAsync(v, final_sums, sizeof v, hipMemcpyDeviceToHost, c->stream), "copy diagnostics");
  HIP_OR_FAIL(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  diag_from_sums(c, v, out);
  return LBM_OK;
}

int lbm_get_dims(lbm_handle h, int* lattice, int64_t dims[3]) {
  if (!h || !lattice || !dims) return fail(LBM_EINVAL, "lbm_get_dims: NULL argument");
  *lattice = h->lattice;
  for (int a = 0; a < 3; ++a) dims[a] = h->n[a];
  return LBM_OK;
}

int lbm_get_tile(lbm_handle h, int tile[3]) {
  if (!h || !tile) return fail(LBM_EINVAL, "lbm_get_tile: NULL argument");
  tile[0] = h->tile.bx;
  tile[1] = h->tile.by;
  tile[2] = h->tile.chunk;
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

static int fields_update(lbm_handle h, const double* drho, const double* du, const double* dT, int mem, bool keep,
                         const char* name) {
  if (!h) return fail(LBM_EINVAL, std::string(name) + ": NULL handle");
  if (!drho || !du || !dT) return fail(LBM_EINVAL, std::string(name) + ": NULL field");
  if (mem != LBM_HOST && mem != LBM_DEVICE) return fail(LBM_EINVAL, std::string(name) + ": bad memory kind");
  Ctx* c = h;
  if (!c->initialised) return fail(LBM_ESTATE, std::string(name) + ": no state (lbm_init_fields)");
  int rc = select_device(c);
  if (rc) return rc;
  if ((rc = ensure_scratch(c))) return rc;
  const int64_t N = c->N;
  const int D = c->lattice;
  if (!c->work) HIP_OR_FAIL(hipMalloc(&c->work, sizeof(double) * 10 * (size_t)N), "hipMalloc(work)");
  double* newf = c->work;
  if (mem == LBM_HOST) {
    double* st = c->work + 5 * N;
    HIP_OR_FAIL(hipMemcpyAsync(st, drho, sizeof(double) * N, hipMemcpyHostToDevice, c->stream), "copy drho");
    HIP_OR_FAIL(hipMemcpyAsync(st + N, du, sizeof(double) * N * D, hipMemcpyHostToDevice, c->stream), "copy du");
    HIP_OR_FAIL(hipMemcpyAsync(st + 4 * N, dT, sizeof(double) * N, hipMemcpyHostToDevice, c->stream), "copy dT");
    drho = st;
    du = st + N;
    dT = st + 4 * N;
  }
  HIP_OR_FAIL(lbm::launch_fields(*c, c->buf[c->cur], c->fields), "moments kernel");
  HIP_OR_FAIL(lbm::launch_fields_plus(*c, c->fields, drho, du, dT, newf, keep), "increment kernel");
  HIP_OR_FAIL(lbm::launch_validate(*c, newf, newf + N, newf + 4 * N, c->partial, c->partial_blocks, c->diag_dev),
              "validate");
  double bad = 0.0;
  HIP_OR_FAIL(hipMemcpyAsync(&bad, c->diag_dev, sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy count");
  HIP_OR_FAIL(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  if (bad != 0.0) return fail(LBM_EINVAL, std::string(name) + ": non-finite value or rho <= 0 or T <= 0 in the new fields");
  HIP_OR_FAIL(lbm::launch_fields_add(*c, c->buf[c->cur], c->fields, newf), "re-equilibration kernel");
  return LBM_OK;
}

int lbm_fields_add(lbm_handle h, const double* drho, const double* du, const double* dT, int mem) {
  return fields_update(h, drho, du, dT, mem, true, "lbm_fields_add");
}

int lbm_fields_set(lbm_handle h, const double* rho, const double* u, const double* T, int mem) {
  return fields_update(h, rho, u, T, mem, false, "lbm_fields_set");
}

int lbm_filter_moments(lbm_handle h, int factor, double* rho, double* u, double* T, int mem) {
  if (!h) return fail(LBM_EINVAL, "lbm_filter_moments: NULL handle");
  if (!rho || !u || !T) return fail(LBM_EINVAL, "lbm_filter_moments: NULL output");
  if (mem != LBM_HOST && mem != LBM_DEVICE) return fail(LBM_EINVAL, "lbm_filter_moments: bad memory kind");
  Ctx* c = h;
  if (!c->initialised) return fail(LBM_ESTATE, "lbm_filter_moments: no state (lbm_init_fields)");
  const int D = c->lattice;
  if (factor < 1 || c->n[0] % factor || c->n[1] % factor || (D == 3 && c->n[2] % factor))
    return fail(LBM_EINVAL, "lbm_filter_moments: dims not divisible by the factor");
  int rc = select_device(c);
  if (rc) return rc;
  if ((rc = ensure_scratch(c))) return rc;
  const int64_t Nc = (c->n[0] / factor) * (c->n[1] / factor) * (D == 3 ? c->n[2] / factor : 1);
  double *r = rho, *v = u, *t = T;
  if (mem == LBM_HOST) {
    if (!c->work) HIP_OR_FAIL(hipMalloc(&c->work, sizeof(double) * 10 * (size_t)c->N), "hipMalloc(work)");
    r = c->work;
    v = r + Nc;
    t = v + 3 * Nc;
  }
  HIP_OR_FAIL(lbm::launch_fields(*c, c->buf[c->cur], c->fields), "moments kernel");
  HIP_OR_FAIL(lbm::launch_filter(*c, c->fields, factor, r, v, t), "filter kernel");
  if (mem == LBM_HOST) {
    HIP_OR_FAIL(hipMemcpyAsync(rho, r, sizeof(double) * Nc, hipMemcpyDeviceToHost, c->stream), "copy rho");
    HIP_OR_FAIL(hipMemcpyAsync(u, v, sizeof(double) * Nc * D, hipMemcpyDeviceToHost, c->stream), "copy u");
    HIP_OR_FAIL(hipMemcpyAsync(T, t, sizeof(double) * Nc, hipMemcpyDeviceToHost, c->stream), "copy T");
    HIP_OR_FAIL(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  }
  return LBM_OK;
}

int lbm_device_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src) return fail(LBM_EINVAL, "lbm_device_copy: NULL pointer");
  if (bytes % 16) return fail(LBM_EINVAL, "lbm_device_copy: bytes must be a multiple of 16");
  if (((uintptr_t)dst | (uintptr_t)src) % 16) return fail(LBM_EINVAL, "lbm_device_copy: pointers must be 16-byte aligned");
  HIP_OR_FAIL(lbm::launch_copy(dst, src, bytes, static_cast<hipStream_t>(stream)), "copy kernel");
  return LBM_OK;
}


// ---------------------------------------------------------------------------
// Batches: several handles stepped by one launch per step
// ---------------------------------------------------------------------------

}  // extern "C"

namespace {

using Batch = lbm_batch_ctx;

// Step parameters of every box for the batch tile, block offsets, upload of
// the table (synchronous on the caller's stream); drops a captured graph.
int batch_layout(Batch* b) {
  int64_t total = 0;
  for (size_t i = 0; i < b->boxes.size(); ++i) {
    const lbm::Ctx* c = b->boxes[i];
    lbm::Tile t = b->tile;
    const int64_t nm = c->lattice == 3 ? c->n[2] : c->n[1];
    if (t.chunk <= 0) t.chunk = lbm::default_chunk(c->lattice, c->n, t.bx, t.by);
    if (t.chunk > nm) t.chunk = (int)nm;
    lbm::BoxEntry& e = b->host[i];
    fill_step_params(c, t, e.p);
    e.buf[0] = c->buf[0];
    e.buf[1] = c->buf[1];
    e.cur = c->cur;
    e.block_start = (int)total;
    total += e.p.nblocks;
    b->cur_dev[i] = c->cur;
  }
  if (total > INT32_MAX) return fail(LBM_EINVAL, "lbm_batch: too many work-groups");
  b->total_blocks = (int)total;
  HIP_OR_FAIL(hipMemcpyAsync(b->table, b->host.data(), sizeof(lbm::BoxEntry) * b->host.size(), hipMemcpyHostToDevice,
                             b->user_stream),
              "upload box table");
  HIP_OR_FAIL(hipStreamSynchronize(b->user_stream), "hipStreamSynchronize");
  if (b->exec) {
    HIP_OR_FAIL(hipGraphExecDestroy(b->exec), "hipGraphExecDestroy");
    b->exec = nullptr;
    b->graph_steps = 0;
  }
  return LBM_OK;
}

int batch_select_device(Batch* b) {
  int cur = -1;
  HIP_OR_FAIL(hipGetDevice(&cur), "hipGetDevice");
  if (cur != b->device) HIP_OR_FAIL(hipSetDevice(b->device), "hipSetDevice");
  return LBM_OK;
}

// Records graph_steps batched steps on the batch's own stream.
int batch_capture(Batch* b, int graph_steps) {
  if (b->exec) {
    HIP_OR_FAIL(hipGraphExecDestroy(b->exec), "hipGraphExecDestroy");
    b->exec = nullptr;
  }
  HIP_OR_FAIL(hipStreamBeginCapture(b->own_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  hipError_t e = hipSuccess;
  for (int j = 0; j < graph_steps && e == hipSuccess; ++j) e = lbm::launch_batch_step(*b, b->own_stream, j & 1);
  if (e == hipSuccess && (graph_steps & 1)) e = lbm::launch_toggle(*b, b->own_stream);
  hipGraph_t graph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(b->own_stream, &graph);
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(e, "batched step kernel (capture)");
  }
  if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
  e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    b->exec = nullptr;
    return hip_fail(e, "hipGraphInstantiate");
  }
  b->graph_steps = graph_steps;
  return LBM_OK;
}

// Supported shared tiles (bx, by) of a lattice.
std::vector<lbm::Tile> batch_candidates(int D) {
  std::vector<lbm::Tile> v;
  if (D == 3) {
    for (int chunk : {4, 8, 16, 32, 64, 128, 256}) {
      v.push_back({64, 4, chunk});
      v.push_back({32, 8, chunk});
      v.push_back({64, 8, chunk});
    }
  } else {
    for (int bx : {64, 128, 256})
      for (int chunk : {4, 8, 16, 32, 64}) v.push_back({bx, 1, chunk});
  }
  return v;
}

}  // namespace

extern "C" {

int lbm_batch_create(lbm_batch* out, const lbm_handle* boxes, int count) {
  if (!out) return fail(LBM_EINVAL, "lbm_batch_create: out is NULL");
  *out = nullptr;
  if (!boxes || count < 1) return fail(LBM_EINVAL, "lbm_batch_create: need at least one handle");
  for (int i = 0; i < count; ++i) {
    if (!boxes[i]) return fail(LBM_EINVAL, "lbm_batch_create: NULL handle");
    if (boxes[i]->lattice != boxes[0]->lattice || boxes[i]->precision != boxes[0]->precision ||
        boxes[i]->device != boxes[0]->device)
      return fail(LBM_EINVAL, "lbm_batch_create: handles differ in lattice, precision or device");
    if (boxes[i]->sp.caloric)
      return fail(LBM_EINVAL, "lbm_batch_create: handles with a general caloric law (cv_poly) are not batched");
    for (int j = 0; j < i; ++j)
      if (boxes[j] == boxes[i]) return fail(LBM_EINVAL, "lbm_batch_create: a handle appears twice");
  }
  Batch* b = new (std::nothrow) lbm_batch_ctx();
  if (!b) return fail(LBM_ENOMEM, "lbm_batch_create: host allocation failed");
  b->lattice = boxes[0]->lattice;
  b->precision = boxes[0]->precision;
  b->device = boxes[0]->device;
  b->boxes.assign(boxes, boxes + count);
  b->host.resize(count);
  b->cur_dev.assign(count, 0);
  b->user_stream = boxes[0]->stream;
  const lbm::Tile t0 = lbm::default_tile(b->lattice, b->precision, boxes[0]->n);
  b->tile = {t0.bx, t0.by, 0};
  int rc = batch_select_device(b);
  hipError_t e = hipSuccess;
  if (rc == LBM_OK) e = hipMalloc(&b->table, sizeof(lbm::BoxEntry) * (size_t)count);
  if (rc == LBM_OK && e == hipSuccess) e = hipStreamCreateWithFlags(&b->own_stream, hipStreamNonBlocking);
  if (rc == LBM_OK && e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
  if (rc == LBM_OK && e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
  if (rc == LBM_OK && e != hipSuccess) rc = hip_fail(e, "lbm_batch_create");
  if (rc == LBM_OK) rc = batch_layout(b);
  if (rc != LBM_OK) {
    lbm_batch_destroy(b);
    return rc;
  }
  *out = b;
  return LBM_OK;
}

int lbm_batch_destroy(lbm_batch b) {
  if (!b) return LBM_OK;
  (void)batch_select_device(b);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->own_stream) (void)hipStreamSynchronize(b->own_stream);
  if (b->table) (void)hipFree(b->table);
  if (b->own_stream) (void)hipStreamDestroy(b->own_stream);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  delete b;
  return LBM_OK;
}

int lbm_batch_set_stream(lbm_batch b, void* hip_stream) {
  if (!b) return fail(LBM_EINVAL, "lbm_batch_set_stream: NULL batch");
  b->user_stream = static_cast<hipStream_t>(hip_stream);
  return LBM_OK;
}

int lbm_batch_set_tile(lbm_batch b, const int tile[3]) {
  if (!b || !tile) return fail(LBM_EINVAL, "lbm_batch_set_tile: NULL argument");
  const lbm::Tile t{tile[0], b->lattice == LBM_D2Q9 && tile[1] == 0 ? 1 : tile[1], tile[2] < 0 ? -1 : tile[2]};
  if (t.chunk < 0 || !lbm::tile_supported(b->lattice, b->precision, {t.bx, t.by, t.chunk > 0 ? t.chunk : 1}))
    return fail(LBM_EINVAL, "lbm_batch_set_tile: launch tile not available");
  if (b->persistent && !lbm::persistent_supported(t))
    return fail(LBM_EINVAL, "lbm_batch_set_tile: the persistent launch form needs a tile of at most 256 work-items");
  int rc = batch_select_device(b);
  if (rc != LBM_OK) return rc;
  b->tile = t;
  return batch_layout(b);
}

int lbm_batch_set_persistent(lbm_batch b, int on) {
  if (!b) return fail(LBM_EINVAL, "lbm_batch_set_persistent: NULL batch");
  if (on != 0 && on != 1) return fail(LBM_EINVAL, "lbm_batch_set_persistent: on must be 0 or 1");
  if (on == 1 && !lbm::persistent_supported(b->tile))
    return fail(LBM_EINVAL, "lbm_batch_set_persistent: the current tile has more than 256 work-items");
  int rc = batch_select_device(b);
  if (rc != LBM_OK) return rc;
  b->persistent = on == 1;
  return batch_layout(b);  // drops a captured graph
}

int lbm_batch_get_persistent(lbm_batch b) { return b ? (b->persistent ? 1 : 0) : -1; }

int lbm_batch_get_tile(lbm_batch b, int tile[3]) {
  if (!b || !tile) return fail(LBM_EINVAL, "lbm_batch_get_tile: NULL argument");
  tile[0] = b->tile.bx;
  tile[1] = b->tile.by;
  tile[2] = b->tile.chunk;
  return LBM_OK;
}

int lbm_batch_tune(lbm_batch b, int reps, double* best_ms) {
  if (!b) return fail(LBM_EINVAL, "lbm_batch_tune: NULL batch");
  if (reps < 1) return fail(LBM_EINVAL, "lbm_batch_tune: reps must be >= 1");
  for (lbm::Ctx* c : b->boxes)
    if (!c->initialised) return fail(LBM_ESTATE, "lbm_batch_tune: a box has no state (lbm_init_fields)");
  int rc = batch_select_device(b);
  if (rc != LBM_OK) return rc;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  HIP_OR_FAIL(hipEventCreate(&t0), "hipEventCreate");
  hipError_t e = hipEventCreate(&t1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(t0);
    return hip_fail(e, "hipEventCreate");
  }
  // Every timed launch reads each box's current buffer and writes the other
  // one (flip 0, no toggle), so the states are left as they were.
  lbm::Tile best = b->tile;
  bool best_persistent = b->persistent;
  float best_t = -1.0f;
  // every candidate tile in both launch forms
  std::vector<std::pair<lbm::Tile, bool>> cands;
  for (const lbm::Tile& t : batch_candidates(b->lattice))
    if (lbm::tile_supported(b->lattice, b->precision, t)) {
      cands.push_back({t, false});
      if (lbm::persistent_supported(t)) cands.push_back({t, true});
    }
  for (const auto& cand : cands) {
    b->tile = cand.first;
    b->persistent = cand.second;
    if ((rc = batch_layout(b)) != LBM_OK) break;
    if ((e = lbm::launch_batch_step(*b, b->user_stream, 0)) != hipSuccess) break;
    if ((e = hipEventRecord(t0, b->user_stream)) != hipSuccess) break;
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = lbm::launch_batch_step(*b, b->user_stream, 0);
    if (e != hipSuccess || (e = hipEventRecord(t1, b->user_stream)) != hipSuccess) break;
    if ((e = hipEventSynchronize(t1)) != hipSuccess) break;
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) break;
    if (best_t < 0.0f || ms < best_t) {
      best_t = ms;
      best = cand.first;
      best_persistent = cand.second;
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  b->tile = best;
  b->persistent = best_persistent;
  const int rc2 = batch_layout(b);
  if (rc != LBM_OK) return rc;
  if (e != hipSuccess) return hip_fail(e, "lbm_batch_tune");
  if (rc2 != LBM_OK) return rc2;
  if (best_ms) *best_ms = best_t / reps;
  return LBM_OK;
}

int lbm_batch_step(lbm_batch b, int64_t n, int graph_steps) {
  if (!b) return fail(LBM_EINVAL, "lbm_batch_step: NULL batch");
  if (n < 0 || graph_steps < 0) return fail(LBM_EINVAL, "lbm_batch_step: negative count");
  for (lbm::Ctx* c : b->boxes) {
    if (!c->initialised) return fail(LBM_ESTATE, "lbm_batch_step: a box has no state (lbm_init_fields)");
    if (c->unstable) return fail(LBM_EUNSTABLE, "lbm_batch_step: a box is unstable (see lbm_diagnostics)");
  }
  if (n == 0) return LBM_OK;
  int rc = batch_select_device(b);
  if (rc != LBM_OK) return rc;
  // a box stepped on its own since the last batched step: refresh the table
  for (size_t i = 0; i < b->boxes.size(); ++i)
    if (b->boxes[i]->cur != b->cur_dev[i]) {
      if ((rc = batch_layout(b)) != LBM_OK) return rc;
      break;
    }
  hipStream_t s = b->user_stream;
  int64_t done = 0;
  int flips = 0;
  if (graph_steps > 0 && n >= graph_steps) {
    if (!b->exec || b->graph_steps != graph_steps)
      if ((rc = batch_capture(b, graph_steps)) != LBM_OK) return rc;
    HIP_OR_FAIL(hipEventRecord(b->ev_in, s), "hipEventRecord");
    HIP_OR_FAIL(hipStreamWaitEvent(b->own_stream, b->ev_in, 0), "hipStreamWaitEvent");
    const int64_t reps = n / graph_steps;
    for (int64_t r = 0; r < reps; ++r) HIP_OR_FAIL(hipGraphLaunch(b->exec, b->own_stream), "hipGraphLaunch");
    HIP_OR_FAIL(hipEventRecord(b->ev_out, b->own_stream), "hipEventRecord");
    HIP_OR_FAIL(hipStreamWaitEvent(s, b->ev_out, 0), "hipStreamWaitEvent");
    done = reps * graph_steps;
    flips = (int)((graph_steps & 1) * (reps & 1));
  }
  const int64_t rest = n - done;
  for (int64_t j = 0; j < rest; ++j) HIP_OR_FAIL(lbm::launch_batch_step(*b, s, (int)(j & 1)), "batched step kernel");
  if (rest & 1) HIP_OR_FAIL(lbm::launch_toggle(*b, s), "toggle kernel");
  flips ^= (int)(rest & 1);
  for (size_t i = 0; i < b->boxes.size(); ++i) {
    lbm::Ctx* c = b->boxes[i];
    c->cur ^= flips;
    c->step += n;
    b->cur_dev[i] = c->cur;
  }
  return LBM_OK;
}

}  // extern "C"
