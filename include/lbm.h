/*
 * lbm.h - C ABI of the MI355X library for the two-population compressible
 * lattice Boltzmann model of Saadat, Hosseini, Dorschner and Karlin,
 * "Extended lattice Boltzmann model for gas dynamics" (arXiv:2102.09512).
 *
 * One call of lbm_step advances the state by one time step of the kinetic
 * equations (1) (f: mass and momentum, BGK relaxation to the extended
 * equilibrium of Eqs. (28)-(30)) and (2) (g: total energy, relaxation to the
 * equilibrium of Eq. (42) and the quasi-equilibrium of Eqs. (44), (46)), with
 * the anomaly derivative of Sec. III.A computed from the post-streaming
 * moments of the same step.  All of it runs in HIP kernels for gfx950.
 *
 * Conventions
 *   - Lattice units: delta_t = delta_x = 1, R = 1; constant specific heats
 *     C_v = 1/(gamma-1) (Sec. III.A).
 *   - Fields are FP64, node-major, node = x + nx*(y + ny*z).  rho[N], T[N];
 *     u holds D consecutive planes u_x[N], u_y[N] (, u_z[N]).
 *   - Population numbering: c_i = (i%3-1, (i/3)%3-1, (i/9)%3-1), Q = 3^D; the
 *     opposite of i is Q-1-i.
 *   - Every call returns an int: LBM_OK (0) or a negative error code; nothing
 *     aborts or throws across the ABI.  lbm_last_error gives the message of
 *     the last failure on the calling thread.
 *   - Ownership: the handle owns all device population buffers.  The caller
 *     owns every array it passes and keeps it alive until the call returns
 *     (for LBM_DEVICE arrays: until the bound stream has passed the call).
 *     The library keeps no caller pointer.
 *   - Streams: work is ordered on the stream given to lbm_set_stream (default:
 *     the null stream of the device that was current at lbm_create).  Calls
 *     with LBM_HOST arrays and lbm_diagnostics synchronise that stream; the
 *     others are asynchronous.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx* lbm_handle;

/* Lattices: value = D.  D3Q27 is Eq. (8); D2Q9 drops the z factor of the
   product form (Eq. (12)). */
enum { LBM_D2Q9 = 2, LBM_D3Q27 = 3 };
/* Population storage.  LBM_FP32_DEV stores f_i - f^eq_i(rho_ref, u_ref, T_ref)
   and g_i - g^eq_i(rho_ref, u_ref, T_ref) in FP32 and collides in FP32 with
   every quantity in deviation form from that reference state; the collision
   restores its FP32 mass, momentum and energy residuals, and moments and
   diagnostics are FP64.  The reference should be close to the flow's typical
   state (e.g. the free stream): the storage error scales with the size of
   the deviations. */
enum { LBM_FP64 = 0, LBM_FP32_DEV = 1 };
/* Boundaries, per axis (both ends): periodic wrap, or zero-gradient (the
   streaming source and every difference neighbour are clamped to the domain). */
enum { LBM_BC_PERIODIC = 0, LBM_BC_ZERO_GRADIENT = 1 };
/* Where caller arrays live. */
enum { LBM_HOST = 0, LBM_DEVICE = 1 };
/* Discrete derivative of the anomaly: first-order upwind (Sec. III.A) or
   second-order central (Sec. III.D.2). */
enum { LBM_DERIV_UPWIND = 0, LBM_DERIV_CENTRAL = 1 };
enum { LBM_LAYOUT_SLOT_ROWS = 0, LBM_LAYOUT_BLOCKS = 1 };
enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,    /* bad argument or field value */
  LBM_ENOMEM = -2,    /* device allocation failed */
  LBM_EDEVICE = -3,   /* a HIP call failed (message in lbm_last_error) */
  LBM_EUNSTABLE = -4, /* the last diagnostics found non-finite or non-positive rho/T */
  LBM_ESTATE = -5     /* call out of order (e.g. lbm_step before lbm_init_fields) */
};

typedef struct {
  int precision;        /* LBM_FP64 (default) or LBM_FP32_DEV */
  int bc[3];            /* per axis; default LBM_BC_PERIODIC */
  double visc_exponent; /* mu = mu0 (T/T_ref)^visc_exponent (Sec. III.D); 0 = constant mu (default) */
  double T_ref;         /* T_0 of the power law and reference temperature of FP32 deviations; default 1/3 */
  double rho_ref;       /* reference density of FP32 deviations; default 1 */
  int deriv_scheme;     /* LBM_DERIV_UPWIND (default) or LBM_DERIV_CENTRAL */
  int tile[3];          /* launch shape of the step kernel: x width, y width (D3Q27), march chunk; 0 = default
                           (a zero chunk with a given shape: the default chunk for that shape).  Shapes:
                           D3Q27 64x4, 32x8 and, for LBM_FP32_DEV only, 64x8; D2Q9 64, 128, 256 wide */
  double u_ref[3];      /* reference velocity of FP32 deviations (|u_ref_a| < 1); default 0 */
  double cv_poly[3];    /* caloric law (Sec. II.A, Eq. (6)): C_v(T) = cv_poly[0] + cv_poly[1] T + cv_poly[2] T^2,
                           U(T) = its integral from 0, T recovered from U by Newton's method; needs
                           cv_poly[0] > 0 and cv_poly[1], cv_poly[2] >= 0.  All zero (default): the
                           constant C_v = 1/(gamma - 1), and gamma is used for nothing else */
  int layout;           /* device layout of the populations of one march plane (x-y plane for D3Q27,
                           x row for D2Q9), (f_i, g_i) pairs throughout:
                           LBM_LAYOUT_SLOT_ROWS (default): slot i of the plane is one contiguous row of
                           pairs (rows 64-pair aligned, staggered by 64 pairs);
                           LBM_LAYOUT_BLOCKS: 64-node blocks, each holding its Q slots of 64 pairs one
                           after the other.  Results are identical to the last bit; only the memory
                           streams differ (a measurement choice).  The ABI state of lbm_get_state is
                           the same for both. */
} lbm_options;

/* Fills *opt with the defaults above. */
void lbm_default_options(lbm_options* opt);

/* Whole-field sums of the stored state (the post-collision populations;
   moments without streaming, Eqs. (3)-(7)).  mass, momentum and energy are
   the conserved totals of Eqs. (3)-(5); the others are the turbulence
   statistics of Sec. III.D: the kinetic energy, the dilatation (whose mean
   square gives the rms dilatation), the vorticity (enstrophy = half its mean
   square) and the dissipation sum mu(T) |curl u|^2 with the viscosity law of
   Sec. III.D, the velocity and sound-speed sums of the turbulent Mach
   number, and per-axis variances of the velocity and of its gradient (the
   Taylor microscale).  Derivatives are central differences with the same
   wrap/clamp rule as the method.  Every sum is FP64 in a fixed order (wave64
   shuffles, then per-work-group partials, then one fixed-order pass), so a
   repeated call gives the same bits. */
typedef struct {
  int64_t step;
  int64_t nodes;
  double mass;              /* sum rho */
  double momentum[3];       /* sum rho u */
  double energy;            /* sum rho E = sum of all g_i */
  double kinetic_energy;    /* sum rho |u|^2 / 2 */
  double dilatation_sq_sum; /* sum (div u)^2 */
  double u2_sum;            /* sum |u|^2 */
  double cs_sum;            /* sum sqrt(gamma T) */
  double rho2_sum;          /* sum rho^2 */
  double vorticity_sq_sum;  /* sum |curl u|^2 */
  double dissipation_sum;   /* sum mu(T) |curl u|^2 */
  double u_axis_sq_sum[3];  /* sum u_a^2 */
  double du_axis_sq_sum[3]; /* sum (d_a u_a)^2 */
  int64_t nonfinite;        /* nodes with a non-finite rho, u or T */
  int64_t nonpositive;      /* nodes with rho <= 0 or T <= 0 */
} lbm_diag;

/* Creates a simulation on the current HIP device.
   lattice: LBM_D2Q9 or LBM_D3Q27; dims: nx, ny, nz (nz must be 1 for D2Q9);
   gamma > 1 (Eq. (97)); Pr > 0 (Eq. (96)); mu > 0 the dynamic viscosity (at
   T_ref when a power law is set), Eq. (92).  opt may be NULL (defaults).
   Allocates the two population buffers (2 x 2Q x N values).  Limits: each
   dimension up to 2^30, N below 2^31, and the 2Q values of one march plane
   (an x-y plane for D3Q27, an x row for D2Q9) below 4 GiB (D3Q27: about
   9.9 M nodes per plane in FP64, 19.9 M in FP32).  Returns LBM_EINVAL before
   any device work on a bad argument; *out is NULL on error. */
int lbm_create(lbm_handle* out, int lattice, const int64_t dims[3], double gamma, double Pr, double mu,
               const lbm_options* opt);
/* Frees everything the handle owns.  NULL is accepted. */
int lbm_destroy(lbm_handle h);
/* Binds a hipStream_t for all later work of this handle. */
int lbm_set_stream(lbm_handle h, void* hip_stream);
/* Sets f = f^eq(rho,u,T) (Eq. (20)) and g = g^eq(rho,u,T) (Eq. (42)), step = 0.
   The equilibria are evaluated in FP64 for either storage (FP32 storage then
   holds each deviation from the reference state rounded once).
   LBM_EINVAL if any value is non-finite or rho <= 0 or T <= 0 (nothing is
   changed then).  mem: LBM_HOST or LBM_DEVICE. */
int lbm_init_fields(lbm_handle h, const double* rho, const double* u, const double* T, int mem);
/* Advances n >= 0 steps (one fused stream-and-collide launch per step).
   LBM_ESTATE before lbm_init_fields; LBM_EUNSTABLE if the last lbm_diagnostics
   found a bad node. */
int lbm_step(lbm_handle h, int64_t n);
/* rho, u, T of the stored populations (Eqs. (3)-(7) without streaming).  Any
   output pointer may be NULL. */
int lbm_moments(lbm_handle h, double* rho, double* u, double* T, int mem);
/* Synchronous reductions over the stored state (FP64, fixed order) into
   *out (host): the totals of Eqs. (3)-(5) and the statistics of Sec. III.D
   listed at lbm_diag.  Sets the handle's instability flag when a node is
   non-finite or has rho <= 0 or T <= 0 (lbm_step then returns
   LBM_EUNSTABLE).  Allocates a 6 N-double field buffer and the partial sums
   on first use.  LBM_EINVAL on a NULL argument, LBM_ESTATE before
   lbm_init_fields. */
int lbm_diagnostics(lbm_handle h, lbm_diag* out);
/* lbm_diagnostics for callers that cannot allocate device memory (code
   under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc): the same sums into *out (host), formed straight from the
   stored populations by the same arithmetic over the same grid, with no
   field buffer and no allocation.  The block partial sums and the final
   sums live in a library-owned device array of 2048 x 21 + 21 doubles
   (344 KB) on each device, obtained at lbm_create and held until the
   process ends; it covers any grid lbm_create accepts (at most 2048
   partial sums), and a reduction that would need more is refused with
   LBM_EINVAL.  All calls on one device share that array and each call
   overwrites it: calls that overlap on one device (from several host
   threads, or on several streams of the device) race and must be serialised
   by the caller.  Synchronous on the handle's stream.  Sets the instability
   flag as lbm_diagnostics does.  LBM_EINVAL on a NULL argument, LBM_ESTATE
   before lbm_init_fields, LBM_EDEVICE if a HIP call (or the scratch
   address) fails. */
int lbm_diagnostics_noalloc(lbm_handle h, lbm_diag* out);
/* Raw state for checkpoints: 2Q population planes of N values (f then g) in
   the storage type (FP64: double values; FP32_DEV: float deviations). */
size_t lbm_state_bytes(lbm_handle h);
int lbm_get_state(lbm_handle h, void* buf, size_t bytes, int mem);
/* Restores a state written by lbm_get_state of a handle with the same lattice,
   dims and precision; the step counter is set to step. */
int lbm_set_state(lbm_handle h, const void* buf, size_t bytes, int mem, int64_t step);
int64_t lbm_step_count(lbm_handle h);
/* Lattice (LBM_D2Q9 or LBM_D3Q27) and dims {nx, ny, nz} of a handle, as
   given to lbm_create (host outputs).  LBM_EINVAL on a NULL argument. */
int lbm_get_dims(lbm_handle h, int* lattice, int64_t dims[3]);
/* Launch tile {bx, by, chunk} of the handle's step kernel (the default chosen
   at lbm_create, or lbm_options.tile).  LBM_EINVAL on a NULL argument. */
int lbm_get_tile(lbm_handle h, int tile[3]);
/* Message of the last failure on this thread ("" if none).  h is unused. */
const char* lbm_last_error(lbm_handle h);
/* Adds increments to the macroscopic fields of the stored state: with (rho,
   u, T) the moments of the stored populations and (rho', u', T') = (rho +
   drho, u + du, T + dT), f_i += f^eq_i(rho', u', T') - f^eq_i(rho, u, T) and
   likewise g (Eqs. (20), (42)), so the non-equilibrium parts are kept and the
   moments become (rho', u', T').  Arrays as in lbm_init_fields; LBM_EINVAL if
   a new rho or T is not positive (nothing changed then). */
int lbm_fields_add(lbm_handle h, const double* drho, const double* du, const double* dT, int mem);
/* As lbm_fields_add with the new fields given instead of increments: the
   moments become (rho, u, T) and the non-equilibrium parts are kept. */
int lbm_fields_set(lbm_handle h, const double* rho, const double* u, const double* T, int mem);
/* Box filter of the stored moments onto the coarse grid of factor^D times
   fewer nodes (every dim divisible by factor; for D2Q9 the z factor is 1):
   rho_c = mean rho, (rho u)_c = mean rho u, (rho E)_c = mean rho E, and
   u_c = (rho u)_c / rho_c, T_c = ((rho E)_c / rho_c - |u_c|^2 / 2) / C_v, so
   mass, momentum and energy are kept.  Outputs on the coarse grid (node
   order as for the fields). */
int lbm_filter_moments(lbm_handle h, int factor, double* rho, double* u, double* T, int mem);
/* Measurement kernel: the memory-access pattern of one lbm_step alone.
   Each of launches launches runs, with the handle's launch tile, a kernel
   that loads exactly what a step loads (the pull sources of every node, of
   the one-node halo ring and of the planes next to each march chunk),
   exchanges the same values through LDS with the same barriers and stores
   exactly what a step stores, but does no collision: it writes the streamed
   populations, plus about one addition per loaded value so that no load is
   dead.  It reads the current populations and writes the other buffer, so
   the state and the step count are unchanged.  Asynchronous on the handle's
   stream.  Its bytes per node are those of a step, so its time is the
   ceiling a step kernel with this access pattern can reach.  LBM_EINVAL on
   a NULL handle, launches < 0 or a handle with cv_poly; LBM_ESTATE before
   lbm_init_fields. */
int lbm_pattern_reference(lbm_handle h, int64_t launches);
/* Plain device-to-device copy of bytes (multiple of 16) on hip_stream, by the
   library's own vectorised copy kernel: the reference for achievable HBM
   bandwidth and for scaling hardware byte counters. */
int lbm_device_copy(void* dst, const void* src, size_t bytes, void* hip_stream);

/* ---- Batches: independent boxes stepped together ----------------------------
   A batch advances several handles (boxes of any sizes, one lattice and one
   precision, one device) by one kernel launch per time step: the launch's
   work-groups are dealt out over all boxes' tiles through a device table, and
   every box computes exactly what lbm_step would (same kernel body, same
   per-box parameters, so the same result to the last bit for FP32 storage).
   The batch does not own the handles: they stay usable on their own (init,
   moments, diagnostics, checkpoints, lbm_step) and must outlive the batch. */
typedef struct lbm_batch_ctx* lbm_batch;

/* Builds a batch over count >= 1 distinct handles (LBM_EINVAL if they differ
   in lattice, precision or device).  Allocates the device box table.  The
   stream is the first handle's; the shared launch tile is the lattice's
   default with per-box march chunks. */
int lbm_batch_create(lbm_batch* out, const lbm_handle* boxes, int count);
/* Frees the batch (not the handles).  NULL is accepted. */
int lbm_batch_destroy(lbm_batch b);
/* Stream on which lbm_batch_step orders its work (after earlier work on it). */
int lbm_batch_set_stream(lbm_batch b, void* hip_stream);
/* Shared launch tile {bx, by, chunk}: bx, by one of the compiled shapes of the
   lattice (as in lbm_options.tile); chunk > 0 for every box, 0 for each box's
   default chunk with that shape.  LBM_EINVAL if not available.  Drops a
   captured graph. */
int lbm_batch_set_tile(lbm_batch b, const int tile[3]);
int lbm_batch_get_tile(lbm_batch b, int tile[3]);
/* Launch form of the batched step: 0 (default) one work-group per tile; 1 a
   fixed grid of work-groups sized by the kernel's occupancy on the device
   (a few per compute unit), in which each XCD takes one contiguous eighth
   of the tiles and its work-groups loop over them (no work-group waits for
   another).  Both compute the same result to the last bit.  The fixed grid
   exists for tiles of at most 256 work-items: LBM_EINVAL for on = 1 with a
   larger tile (and from lbm_batch_set_tile for such a tile while on = 1),
   and for another value of on.  A batch whose tiles all fit on the device
   at once launches one work-group per tile either way.  Drops a captured
   graph. */
int lbm_batch_set_persistent(lbm_batch b, int on);
/* The launch form in use (0 or 1), -1 for a NULL batch. */
int lbm_batch_get_persistent(lbm_batch b);
/* Autotuner: times every compiled shape with several march-chunk lengths, in
   both launch forms, over reps launches each and keeps the fastest; *best_ms
   (may be NULL) gets its time per step.  The timed launches read each box's current populations and
   write the other buffer only, so the states are unchanged.  Synchronous. */
int lbm_batch_tune(lbm_batch b, int reps, double* best_ms);
/* Advances every box by n >= 0 steps.  graph_steps > 0: the launches of
   graph_steps steps are captured once into a HIP graph (re-captured when
   graph_steps or the tile changes) and replayed n / graph_steps times; the
   remaining steps are launched directly.  Asynchronous.  LBM_ESTATE if a box
   has no state, LBM_EUNSTABLE if a box's last diagnostics found a bad node. */
int lbm_batch_step(lbm_batch b, int64_t n, int graph_steps);

#ifdef __cplusplus
}
#endif
#endif
