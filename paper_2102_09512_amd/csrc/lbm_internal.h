// Internal declarations shared by the host API and the kernel launchers of
// liblbm.so.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "lbm.h"

namespace lbm {

// Everything the step kernel needs, passed by value.
struct StepParams {
  int nx, ny, nz;
  int bc[3];            // LBM_BC_* per axis
  // Layout of one march plane: in-plane node q sits in 64-node block q / 64
  // at lane q % 64; element (f or g) s of slot i is at
  //   (q / 64) * blk + i * sl + 2 (q % 64) + s.
  long long sl;         // elements between the same block of two consecutive slots
  long long blk;        // elements between two consecutive 64-node blocks of one slot
  long long ms;         // elements between two consecutive march planes (z for D3Q27, y for D2Q9)
  int plane;            // nodes per march plane (nx*ny for D3Q27, nx for D2Q9)
  int tiles_x, tiles_y; // in-plane tiles (tiles_y == 1 for D2Q9)
  int chunks, chunk_len;// march-axis chunks (z for D3Q27, y for D2Q9)
  int nblocks;
  int deriv;            // LBM_DERIV_*
  // Reference state (rho0, u0, T0) of the FP32 deviation storage; all zero
  // for FP64 storage.  rhoE0 = rho0 (U(T0) + |u0|^2/2) and j0 = rho0 u0 are
  // the reference's energy and momentum; P0, psi0, b0 the per-axis factors
  // of its product-form populations (see NodeConsts).
  double rho0, T0, rhoE0;
  double u0[3], j0[3], P0[3], psi0[3][3], b0[3][3];
  float u0f[3], P0f[3], psi0f[3][3], b0f[3][3];
  // Caloric law: C_v(T) = Cv + cv1 T + cv2 T^2 when caloric != 0, else the
  // constant Cv; U0 = U(T0).
  double Cv, inv_Cv, Pr;
  double cv1, cv2, U0;
  int caloric;
  double mu0, visc_exp, inv_Tref;
  double gamma;
};

// Caloric law (Eq. (6)): C_v(T) = c0 + c1 T + c2 T^2 and U(T) its integral
// from 0.
__host__ __device__ inline double caloric_cv(double c0, double c1, double c2, double T) { return c0 + T * (c1 + T * c2); }
__host__ __device__ inline double caloric_u(double c0, double c1, double c2, double T) {
  return T * (c0 + T * (0.5 * c1 + T * (c2 / 3.0)));
}

// Launch shape of the step kernel (compile-time instantiations).
struct Tile {
  int bx, by, chunk;
};

struct Ctx {
  int lattice = 0;      // D
  int Q = 0;
  int precision = 0;
  int64_t n[3] = {1, 1, 1};
  int64_t N = 0;
  long long sl = 0;       // slot stride inside a plane (see StepParams)
  long long blk = 0;      // 64-node block stride inside a plane
  long long ms = 0;       // march-plane stride
  int nm = 0;             // number of march planes
  int device = 0;
  hipStream_t stream = nullptr;
  double gamma = 1.4, Pr = 0.71, mu = 0.01;
  lbm_options opt{};
  Tile tile{};
  void* buf[2] = {nullptr, nullptr}; // population buffers (2Q x ps elements each)
  int cur = 0;                       // buffer holding the current state
  double* fields = nullptr;          // 6 x N doubles: rho, ux, uy, uz, T, rhoE
  double* work = nullptr;            // 10 x N doubles, on first use: new fields and staged increments
  double* partial = nullptr;         // per-block partial sums
  double* diag_dev = nullptr;        // final sums
  int partial_blocks = 0;
  bool initialised = false;
  bool unstable = false;
  int64_t step = 0;
  StepParams sp{};
};

constexpr int kNumDiag = 21;  // slots of the diagnostic reduction (see lbm_kernels.hip)
constexpr int kMaxDiagBlocks = 2048;  // work-groups of a diagnostic reduction, at most
// doubles of the allocation-free diagnostics' device scratch: the block
// partials of the largest grid, then the final sums
constexpr int kScratchDoubles = kMaxDiagBlocks * kNumDiag + kNumDiag;

// One box of a batched launch (an entry of the device box table).
struct BoxEntry {
  StepParams p;       // the box's step parameters for the batch tile
  void* buf[2];       // the box's population buffers
  int cur;            // buffer holding the box's state when the launch sequence starts
  int block_start;    // first logical work-group of the box in the launch
};

// Several handles of one lattice and precision stepped by one launch per step.
struct Batch {
  int lattice = 0, precision = 0, device = 0;
  std::vector<Ctx*> boxes;
  std::vector<BoxEntry> host;      // host image of the table
  BoxEntry* table = nullptr;       // device table
  std::vector<int> cur_dev;        // cur of each box as the device table holds it
  int total_blocks = 0;
  Tile tile{};                     // bx, by shared by all boxes; chunk 0 = per-box default
  bool persistent = false;         // fixed grid looping over the tiles instead of one work-group per tile
  hipStream_t user_stream = nullptr;
  hipStream_t own_stream = nullptr;  // graph replays run here
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t exec = nullptr;     // captured sequence of graph_steps steps
  int graph_steps = 0;
};

// ---- launchers (lbm_kernels.hip) -------------------------------------------
hipError_t launch_step(const Ctx& c, const void* src, void* dst);
// The step kernel's access pattern without the node arithmetic (measurement).
hipError_t launch_pattern(const Ctx& c, const void* src, void* dst);
hipError_t launch_init(const Ctx& c, const double* rho, const double* u, const double* T, void* dst);
hipError_t launch_fields(const Ctx& c, const void* pops, double* fields);
hipError_t launch_diag(const Ctx& c, const double* fields, double* partial, int nblocks, double* out);
// The same sums straight from the populations (no field buffer), and the
// device address of the current device's allocation-free scratch
// (kScratchDoubles doubles).
hipError_t launch_diag_direct(const Ctx& c, const void* pops, double* partial, int nblocks, double* out);
hipError_t scratch_address(double** out);
int diag_blocks(const Ctx& c);
hipError_t launch_validate(const Ctx& c, const double* rho, const double* u, const double* T, double* partial,
                           int nblocks, double* out);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
// Internal population layout <-> the ABI state layout (2Q arrays of N values).
hipError_t launch_pack(const Ctx& c, const void* pops, void* state);
hipError_t launch_unpack(const Ctx& c, const void* state, void* pops);
// Records msg as the calling thread's last error (lbm_last_error); returns code.
int set_error(int code, const std::string& msg);
hipError_t launch_fields_add(const Ctx& c, void* pops, const double* oldf, const double* newf);
hipError_t launch_fields_plus(const Ctx& c, const double* oldf, const double* drho, const double* du, const double* dT,
                              double* newf, bool keep);
hipError_t launch_filter(const Ctx& c, const double* fields, int factor, double* rho, double* u, double* T);
// Corrector support (host, lbm_api.hip): moments into c->fields; increments
// applied by re-equilibration, asynchronously and without validation.
int fields_current(Ctx* c);
int fields_increment_async(Ctx* c, const double* drho, const double* du, const double* dT);
hipError_t launch_batch_step(const Batch& b, hipStream_t s, int flip);
hipError_t launch_toggle(const Batch& b, hipStream_t s);
// Default launch tile for a lattice/precision, the default march chunk for a
// given shape, and whether a tile is available.
Tile default_tile(int D, int precision, const int64_t n[3], bool caloric = false);
int default_chunk(int D, const int64_t n[3], int bx, int by);
bool tile_supported(int D, int precision, const Tile& t, bool caloric = false);
// Whether the persistent form of the batched launch exists for a tile.
bool persistent_supported(const Tile& t);

}  // namespace lbm

// The opaque handle type of the C ABI.
struct lbm_ctx : public lbm::Ctx {};
struct lbm_batch_ctx : public lbm::Batch {};
