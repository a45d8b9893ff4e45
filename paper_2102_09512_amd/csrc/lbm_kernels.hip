// HIP kernels of liblbm.so (gfx950).
//
// Fused stream-and-collide (one launch per time step)
// ---------------------------------------------------
// Populations are stored plane-major structure-of-arrays: for every plane of
// the march axis (z for D3Q27, y for D2Q9) the 2Q populations of that plane
// follow each other, each as one contiguous in-plane array (x fastest):
//   buf[m * ms + i * ps + p],  p = in-plane node index, f first (i < Q),
//   g after (Q <= i < 2Q).
// A work-group that marches over a few planes then touches a few MB of
// address space instead of 2Q arrays a whole field apart, which keeps the
// address translation caches warm.
// Streaming is done by pull: the thread of node x reads population i from
// x - c_i (wrapped or clamped per axis) and writes the post-collision values
// at x, so every store of a wavefront is a contiguous 256-byte (FP32) or
// 512-byte (FP64) run.
//
// The anomaly correction needs, at node x, the post-streaming anomaly Qt_a of
// the neighbours x +- e_a of the same step.  A work-group owns a BX x BY tile
// of an in-plane slab and marches along the last axis (z for D3Q27, y for
// D2Q9) over a chunk of planes:
//   - each thread keeps its own node's post-streaming populations in
//     registers from the plane where they are loaded (m + 1) to the plane where
//     they are collided (m); the neighbours along the march axis are the
//     same thread's previous and next planes, held in registers;
//   - neighbours inside the plane are exchanged through LDS; a one-node ring
//     around the tile (the halo) is computed by the first threads of the
//     group, which pull the halo nodes' populations and form their moments
//     (these re-reads mostly hit L2: the halo is the neighbouring tile's core);
//   - one barrier per plane.
// Work-groups are mapped XCD-aware: consecutive hardware block ids go to
// different XCDs, so the logical tile order is rebuilt such that every XCD
// processes one contiguous range of tiles (neighbouring tiles share an L2).
#include <hip/hip_runtime.h>

#include "lbm_internal.h"
#include "lbm_node.h"

namespace lbm {

__device__ inline int fix_coord(int k, int n, int bc) {
  if (bc == LBM_BC_PERIODIC) {
    k %= n;
    return k < 0 ? k + n : k;
  }
  return k < 0 ? 0 : (k > n - 1 ? n - 1 : k);
}

// Element offset of population i of node n (node = x + nx*(y + ny*z)).
__device__ inline long long pop_offset(const StepParams& p, int i, long long n) {
  const long long m = n / p.plane;
  return m * p.ms + (long long)i * p.ps + (n - m * p.plane);
}

template <typename S>
struct StoreOf;
template <>
struct StoreOf<float> {
  using R = float;
};
template <>
struct StoreOf<double> {
  using R = double;
};

__device__ inline NodeConsts node_consts(const StepParams& p) {
  NodeConsts k;
  k.rho0 = p.rho0;
  k.T0 = p.T0;
  k.inv_Cv = p.inv_Cv;
  k.Cv = p.Cv;
  k.Pr = p.Pr;
  k.mu0 = p.mu0;
  k.visc_exp = p.visc_exp;
  k.inv_Tref = p.inv_Tref;
  return k;
}

// Raw buffer access: a wave-uniform resource (base of one march plane), a
// per-lane 32-bit byte offset (the in-plane node) and a wave-uniform scalar
// offset (the population), so a load or store needs no per-lane address
// arithmetic.  Offsets past the resource's size read 0 and drop writes.
constexpr int kBufferFlags = 0x00020000;  // raw 32-bit data format (gfx9 family)

__device__ inline __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, long long bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufferFlags);
}

template <typename S>
struct Buf;
template <>
struct Buf<float> {
  static __device__ inline float load(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
  }
  static __device__ inline void store(float v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, 0);
  }
};
template <>
struct Buf<double> {
  static __device__ inline double load(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
  }
  static __device__ inline void store(double v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, vo, so, 0);
  }
};

// Pull-load the 2Q populations arriving at a node.  rs[k] is the resource of
// march plane (m + k - 1) after wrap/clamp; lo[j] is the byte offset inside a
// plane of the in-plane source (y + j/3 - 1, x + j%3 - 1).  Population i of
// the source x - c_i sits at scalar offset i * ps_bytes of plane 1 - c_m.
template <int D, typename S, typename R>
__device__ inline void pull(const __amdgpu_buffer_rsrc_t* rs, unsigned ps_bytes, const unsigned* lo, R* f, R* g) {
  constexpr int Q = lat_q(D);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = vx(i);
    const int cy = (D == 3) ? vy(i) : 0;
    const int cm = (D == 3) ? vz(i) : vy(i);
    const unsigned o = lo[(1 - cy) * 3 + (1 - cx)];
    f[i] = (R)Buf<S>::load(rs[1 - cm], o, (unsigned)i * ps_bytes);
    g[i] = (R)Buf<S>::load(rs[1 - cm], o, (unsigned)(i + Q) * ps_bytes);
  }
}

template <int D, bool DEV, typename S, int BX, int BY>
__global__ void __launch_bounds__(BX* BY) step_kernel(const S* __restrict__ src, S* __restrict__ dst,
                                                      const StepParams p) {
  using R = typename StoreOf<S>::R;
  constexpr int Q = lat_q(D);
  constexpr int NHALO = (D == 3) ? 2 * BX + 2 * BY : 2;
  static_assert(BX * BY >= NHALO, "tile too small for its halo");
  static_assert(D == 3 || BY == 1, "D2Q9 tiles are one row");
  __shared__ R lq0[2][BY][BX + 2];                    // anomaly along in-plane axis 0 (x)
  __shared__ R lq1[2][(D == 3) ? BY + 2 : 1][BX];     // anomaly along in-plane axis 1 (y, D3Q27 only)

  const NodeConsts k = node_consts(p);

  // XCD-aware logical block
  const int b = blockIdx.x;
  const int q8 = p.nblocks >> 3, r8 = p.nblocks & 7, xcd = b & 7;
  const int lb = xcd * q8 + min(xcd, r8) + (b >> 3);
  const int tx = lb % p.tiles_x;
  const int rest = lb / p.tiles_x;
  const int ty = (D == 3) ? rest % p.tiles_y : 0;
  const int ck = (D == 3) ? rest / p.tiles_y : rest;

  const int n0 = p.nx;
  const int n1 = (D == 3) ? p.ny : 1;
  const int nm = (D == 3) ? p.nz : p.ny;
  const int bc0 = p.bc[0], bc1 = p.bc[1], bcm = (D == 3) ? p.bc[2] : p.bc[1];
  const long long sm = p.ms;  // march-plane stride
  const long long ps = p.ps;

  const int t = threadIdx.x;
  const int lx = t % BX, ly = t / BX;
  const int x0 = tx * BX, y0 = ty * BY;
  const int m0 = ck * p.chunk_len;
  const int m1 = min(m0 + p.chunk_len, nm);

  // core node of this thread (positions beyond the domain map by wrap/clamp)
  const int gx = x0 + lx, gy = y0 + ly;
  const bool active = gx < n0 && gy < n1;
  // A position outside the domain stands for the node it maps to, so the
  // neighbour offsets are taken around that node (this matters for clamping).
  int cox[3], coy[3];
  const int gxn = fix_coord(gx, n0, bc0), gyn = fix_coord(gy, n1, bc1);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    cox[j] = fix_coord(gxn + j - 1, n0, bc0);
    coy[j] = (D == 3) ? fix_coord(gyn + j - 1, n1, bc1) * p.nx : 0;
  }
  const int cnode = cox[1] + coy[1];

  // halo node of this thread, if any
  const bool has_halo = t < NHALO;
  int hx = 0, hy = 0, hslot = 0;  // hslot: 0 y-low, 1 y-high, 2 x-low, 3 x-high
  if (D == 3) {
    if (t < BX) {
      hx = x0 + t, hy = y0 - 1, hslot = 0;
    } else if (t < 2 * BX) {
      hx = x0 + t - BX, hy = y0 + BY, hslot = 1;
    } else if (t < 2 * BX + BY) {
      hx = x0 - 1, hy = y0 + t - 2 * BX, hslot = 2;
    } else {
      hx = x0 + BX, hy = y0 + t - 2 * BX - BY, hslot = 3;
    }
  } else {
    hx = (t == 0) ? x0 - 1 : x0 + BX;
    hy = 0;
    hslot = (t == 0) ? 2 : 3;
  }
  int hox[3], hoy[3];
  const int hxn = fix_coord(hx, n0, bc0), hyn = fix_coord(hy, n1, bc1);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    hox[j] = fix_coord(hxn + j - 1, n0, bc0);
    hoy[j] = (D == 3) ? fix_coord(hyn + j - 1, n1, bc1) * p.nx : 0;
  }

  const unsigned psb = (unsigned)(ps * (long long)sizeof(S));
  const long long plane_bytes = sm * (long long)sizeof(S);
  // byte offsets of the 9 in-plane sources of the core and of the halo node
  unsigned clo[9], hlo[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    clo[j] = (unsigned)(sizeof(S) * (unsigned)(coy[j / 3] + cox[j % 3]));
    hlo[j] = (unsigned)(sizeof(S) * (unsigned)(hoy[j / 3] + hox[j % 3]));
  }
  auto march_planes = [&](int m, __amdgpu_buffer_rsrc_t* rs) {
    const int mn = fix_coord(m, nm, bcm);
#pragma unroll
    for (int j = 0; j < 3; ++j) rs[j] = plane_rsrc(src + (long long)fix_coord(mn + j - 1, nm, bcm) * sm, plane_bytes);
  };

  // Post-streaming moments of the halo node at plane m -> LDS buffer.
  auto halo_plane = [&](int m, int buf) {
    if (!has_halo) return;
    __amdgpu_buffer_rsrc_t rs[3];
    march_planes(m, rs);
    R f[Q], g[Q];
    pull<D, S, R>(rs, psb, hlo, f, g);
    NodeMoments<R> mm;
    if constexpr (DEV) mm = node_moments_light<D>(f, g, k);
    else mm = node_moments<D, R>(f, g, k);
    if (D == 3) {
      if (hslot == 0) lq1[buf][0][t] = anomaly(mm, 1);
      else if (hslot == 1) lq1[buf][BY + 1][t - BX] = anomaly(mm, 1);
      else if (hslot == 2) lq0[buf][t - 2 * BX][0] = anomaly(mm, 0);
      else lq0[buf][t - 2 * BX - BY][BX + 1] = anomaly(mm, 0);
    } else {
      lq0[buf][0][hslot == 2 ? 0 : BX + 1] = anomaly(mm, 0);
    }
  };

  // prologue: anomaly along the march axis at plane m0 - 1 (core only)
  R qm_prev, qm_cur, qm_next;
  R fa[Q], ga[Q];
  NodeMoments<R> ma;
  {
    __amdgpu_buffer_rsrc_t rs[3];
    march_planes(m0 - 1, rs);
    pull<D, S, R>(rs, psb, clo, fa, ga);
    NodeMoments<R> mm;
    if constexpr (DEV) mm = node_moments_light<D>(fa, ga, k);
    else mm = node_moments<D, R>(fa, ga, k);
    qm_prev = anomaly(mm, D - 1);
  }
  // plane m0: core populations stay in registers, in-plane anomaly to LDS
  {
    __amdgpu_buffer_rsrc_t rs[3];
    march_planes(m0, rs);
    pull<D, S, R>(rs, psb, clo, fa, ga);
    ma = node_moments<D, R>(fa, ga, k);
    qm_cur = anomaly(ma, D - 1);
    lq0[0][ly][lx + 1] = anomaly(ma, 0);
    if (D == 3) lq1[0][ly + 1][lx] = anomaly(ma, 1);
    halo_plane(m0, 0);
  }
  __syncthreads();

  for (int m = m0; m < m1; ++m) {
    const int cb = (m - m0) & 1, nb = cb ^ 1;
    // load plane m + 1 (core and halo), its moments and anomalies
    R fb[Q], gb[Q];
    NodeMoments<R> mb;
    {
      __amdgpu_buffer_rsrc_t rs[3];
      march_planes(m + 1, rs);
      pull<D, S, R>(rs, psb, clo, fb, gb);
      mb = node_moments<D, R>(fb, gb, k);
      qm_next = anomaly(mb, D - 1);
      lq0[nb][ly][lx + 1] = anomaly(mb, 0);
      if (D == 3) lq1[nb][ly + 1][lx] = anomaly(mb, 1);
      halo_plane(m + 1, nb);
    }
    // collide plane m
    R dd[3];
    dd[0] = anomaly_derivative<R>(p.deriv, ma.u[0], lq0[cb][ly][lx], lq0[cb][ly][lx + 1], lq0[cb][ly][lx + 2]);
    if (D == 3) {
      dd[1] = anomaly_derivative<R>(p.deriv, ma.u[1], lq1[cb][ly][lx], lq1[cb][ly + 1][lx], lq1[cb][ly + 2][lx]);
      dd[2] = anomaly_derivative<R>(p.deriv, ma.u[2], qm_prev, qm_cur, qm_next);
    } else {
      dd[1] = anomaly_derivative<R>(p.deriv, ma.u[1], qm_prev, qm_cur, qm_next);
      dd[2] = (R)0;
    }
    collide<D, R, DEV>(fa, ga, ma, dd, k);
    if (active) {
      const __amdgpu_buffer_rsrc_t rd = plane_rsrc(dst + (long long)m * sm, plane_bytes);
      const unsigned o = (unsigned)(sizeof(S) * (unsigned)cnode);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        Buf<S>::store((S)fa[i], rd, o, (unsigned)i * psb);
        Buf<S>::store((S)ga[i], rd, o, (unsigned)(i + Q) * psb);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      fa[i] = fb[i];
      ga[i] = gb[i];
    }
    ma = mb;
    qm_prev = qm_cur;
    qm_cur = qm_next;
  }
}

// ---------------------------------------------------------------------------
// Initialisation: f = f^eq, g = g^eq (minus the rest state when DEV)
// ---------------------------------------------------------------------------

template <int D, bool DEV, typename S>
__global__ void __launch_bounds__(256) init_kernel(const double* __restrict__ rho, const double* __restrict__ u,
                                                   const double* __restrict__ T, S* __restrict__ dst, long long N,
                                                   const StepParams p) {
  using R = typename StoreOf<S>::R;
  constexpr int Q = lat_q(D);
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const NodeConsts k = node_consts(p);
  NodeMoments<R> m;
  const double r = rho[n], tt = T[n];
  m.rho = (R)r;
  m.drho = (R)(r - p.rho0);
  m.T = (R)tt;
  m.dT = (R)(tt - p.T0);
  m.u[0] = (R)u[n];
  m.u[1] = (R)u[N + n];
  m.u[2] = (D == 3) ? (R)u[2 * N + n] : (R)0;
  m.omega = (R)1;  // corr = (2 - omega)/(2 rho omega) multiplies d = 0
  m.omega1 = (R)1;
  R d[3] = {0, 0, 0};
  R fe[Q], ge[Q];
  equilibria<D, R, DEV>(m, d, k, fe, ge);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    dst[pop_offset(p, i, n)] = (S)fe[i];
    dst[pop_offset(p, i + Q, n)] = (S)ge[i];
  }
}

// ---------------------------------------------------------------------------
// Moments of the stored populations (no streaming), FP64 fields
// fields: rho, ux, uy, uz, T, rhoE (each N)
// ---------------------------------------------------------------------------

template <int D, bool DEV, typename S>
__global__ void __launch_bounds__(256) fields_kernel(const S* __restrict__ pops, double* __restrict__ fields,
                                                     long long N, const StepParams p) {
  constexpr int Q = lat_q(D);
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  double s0 = 0, jx = 0, jy = 0, jz = 0, se = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double v = (double)pops[pop_offset(p, i, n)];
    s0 += v;
    se += (double)pops[pop_offset(p, i + Q, n)];
    const int cx = vx(i), cy = vy(i), cz = (D == 3) ? vz(i) : 0;
    if (cx) jx += cx > 0 ? v : -v;
    if (cy) jy += cy > 0 ? v : -v;
    if (cz) jz += cz > 0 ? v : -v;
  }
  const double rho = p.rho0 + s0;
  const double ux = jx / rho, uy = jy / rho, uz = (D == 3) ? jz / rho : 0.0;
  const double rhoE = p.rhoE0 + se;
  const double T = (rhoE / rho - 0.5 * (ux * ux + uy * uy + uz * uz)) * p.inv_Cv;
  fields[n] = rho;
  fields[N + n] = ux;
  fields[2 * N + n] = uy;
  fields[3 * N + n] = uz;
  fields[4 * N + n] = T;
  fields[5 * N + n] = rhoE;
}

// ---------------------------------------------------------------------------
// Reductions: wave64 shuffles, then LDS across the waves of a block, FP64
// per-block partials; a one-block pass sums the partials in a fixed order.
// ---------------------------------------------------------------------------

template <int NV>
__device__ inline void block_reduce_store(double (&v)[NV], double* __restrict__ out) {
  __shared__ double red[NV][4];  // 256 threads = 4 waves
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    double x = v[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    v[j] = x;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) red[j][wave] = v[j];
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    const int j = threadIdx.x;
    out[j] = (red[j][0] + red[j][1]) + (red[j][2] + red[j][3]);
  }
}

__device__ inline int fix_node_axis(int k, int n, int bc) { return fix_coord(k, n, bc); }

template <int D>
__global__ void __launch_bounds__(256) diag_kernel(const double* __restrict__ F, double* __restrict__ partial,
                                                   long long N, const StepParams p) {
  double acc[kNumDiag];
#pragma unroll
  for (int j = 0; j < kNumDiag; ++j) acc[j] = 0.0;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(n % nx);
    const int y = (int)((n / nx) % ny);
    const int z = (int)(n / ((long long)nx * ny));
    auto at = [&](int comp, int xx, int yy, int zz) {
      return F[(long long)comp * N + xx + (long long)nx * (yy + (long long)ny * zz)];
    };
    const int xp = fix_node_axis(x + 1, nx, p.bc[0]), xm = fix_node_axis(x - 1, nx, p.bc[0]);
    const int yp = fix_node_axis(y + 1, ny, p.bc[1]), ym = fix_node_axis(y - 1, ny, p.bc[1]);
    const int zp = fix_node_axis(z + 1, nz, p.bc[2]), zm = fix_node_axis(z - 1, nz, p.bc[2]);
    const double rho = F[n], ux = F[N + n], uy = F[2 * N + n], uz = F[3 * N + n], T = F[4 * N + n],
                 rhoE = F[5 * N + n];
    // central differences d_b u_a
    const double dxux = 0.5 * (at(1, xp, y, z) - at(1, xm, y, z));
    const double dyuy = 0.5 * (at(2, x, yp, z) - at(2, x, ym, z));
    const double dzuz = (D == 3) ? 0.5 * (at(3, x, y, zp) - at(3, x, y, zm)) : 0.0;
    const double dxuy = 0.5 * (at(2, xp, y, z) - at(2, xm, y, z));
    const double dyux = 0.5 * (at(1, x, yp, z) - at(1, x, ym, z));
    double wx = 0.0, wy = 0.0;
    if (D == 3) {
      wx = 0.5 * (at(3, x, yp, z) - at(3, x, ym, z)) - 0.5 * (at(2, x, y, zp) - at(2, x, y, zm));
      wy = 0.5 * (at(1, x, y, zp) - at(1, x, y, zm)) - 0.5 * (at(3, xp, y, z) - at(3, xm, y, z));
    }
    const double wz = dxuy - dyux;
    const double vort2 = wx * wx + wy * wy + wz * wz;
    const double div = dxux + dyuy + dzuz;
    const double uu = ux * ux + uy * uy + uz * uz;
    const bool finite = isfinite(rho) && isfinite(T) && isfinite(ux) && isfinite(uy) && isfinite(uz);
    const double mu = (p.visc_exp == 0.0) ? p.mu0 : p.mu0 * pow(T * p.inv_Tref, p.visc_exp);
    acc[0] += rho;
    acc[1] += rho * ux;
    acc[2] += rho * uy;
    acc[3] += rho * uz;
    acc[4] += rhoE;
    acc[5] += 0.5 * rho * uu;
    acc[6] += div * div;
    acc[7] += uu;
    acc[8] += sqrt(p.gamma * T);
    acc[9] += rho * rho;
    acc[10] += vort2;
    acc[11] += mu * vort2;
    acc[12] += ux * ux;
    acc[13] += uy * uy;
    acc[14] += uz * uz;
    acc[15] += dxux * dxux;
    acc[16] += dyuy * dyuy;
    acc[17] += dzuz * dzuz;
    acc[18] += finite ? 0.0 : 1.0;
    acc[19] += (rho <= 0.0 || T <= 0.0) ? 1.0 : 0.0;
    acc[20] += 1.0;
  }
  block_reduce_store<kNumDiag>(acc, partial + (long long)blockIdx.x * kNumDiag);
}

template <int NV>
__global__ void __launch_bounds__(256) final_reduce_kernel(const double* __restrict__ partial, int nblocks,
                                                           double* __restrict__ out) {
  double acc[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] += partial[(long long)b * NV + j];
  }
  block_reduce_store<NV>(acc, out);
}

// Counts nodes of a candidate initial field with non-finite values or
// rho <= 0 or T <= 0 (slot 0).
template <int D>
__global__ void __launch_bounds__(256) validate_kernel(const double* __restrict__ rho, const double* __restrict__ u,
                                                       const double* __restrict__ T, double* __restrict__ partial,
                                                       long long N) {
  double acc[1] = {0.0};
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
    bool ok = isfinite(rho[n]) && isfinite(T[n]) && rho[n] > 0.0 && T[n] > 0.0;
    for (int a = 0; a < D; ++a) ok = ok && isfinite(u[(long long)a * N + n]);
    acc[0] += ok ? 0.0 : 1.0;
  }
  block_reduce_store<1>(acc, partial + blockIdx.x);
}

__global__ void __launch_bounds__(256) copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                   long long n16) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

template <typename S>
__global__ void __launch_bounds__(256) pack_kernel(const S* __restrict__ pops, S* __restrict__ state, long long N,
                                                   int nq, const StepParams p) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  for (int i = 0; i < nq; ++i) state[(long long)i * N + n] = pops[pop_offset(p, i, n)];
}

template <typename S>
__global__ void __launch_bounds__(256) unpack_kernel(const S* __restrict__ state, S* __restrict__ pops, long long N,
                                                     int nq, const StepParams p) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  for (int i = 0; i < nq; ++i) pops[pop_offset(p, i, n)] = state[(long long)i * N + n];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

template <int D, bool DEV, typename S, int BX, int BY>
static hipError_t launch_step_t(const Ctx& c, const void* src, void* dst) {
  hipLaunchKernelGGL((step_kernel<D, DEV, S, BX, BY>), dim3(c.sp.nblocks), dim3(BX * BY), 0, c.stream,
                     static_cast<const S*>(src), static_cast<S*>(dst), c.sp);
  return hipGetLastError();
}

// Compiled launch shapes: (D, precision) -> {BX, BY}; the march chunk is a
// runtime parameter.
Tile default_tile(int D, int precision, const int64_t n[3]) {
  if (D == 3) {
    if (precision == LBM_FP64) return Tile{64, 8, (int)(n[2] < 32 ? n[2] : 32)};
    return Tile{64, 8, (int)(n[2] < 64 ? n[2] : 64)};
  }
  return Tile{128, 1, (int)(n[1] < 32 ? n[1] : 32)};
}

bool tile_supported(int D, int precision, const Tile& t) {
  (void)precision;
  if (D == 3) return (t.bx == 64 && (t.by == 4 || t.by == 8)) || (t.bx == 32 && t.by == 8);
  return t.by == 1 && (t.bx == 64 || t.bx == 128 || t.bx == 256);
}

template <int D, bool DEV, typename S>
static hipError_t dispatch_tile(const Ctx& c, const void* src, void* dst) {
  const Tile& t = c.tile;
  if constexpr (D == 3) {
    if (t.bx == 64 && t.by == 4) return launch_step_t<D, DEV, S, 64, 4>(c, src, dst);
    if (t.bx == 64 && t.by == 8) return launch_step_t<D, DEV, S, 64, 8>(c, src, dst);
    if (t.bx == 32 && t.by == 8) return launch_step_t<D, DEV, S, 32, 8>(c, src, dst);
  } else {
    if (t.bx == 64) return launch_step_t<D, DEV, S, 64, 1>(c, src, dst);
    if (t.bx == 128) return launch_step_t<D, DEV, S, 128, 1>(c, src, dst);
    if (t.bx == 256) return launch_step_t<D, DEV, S, 256, 1>(c, src, dst);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_step(const Ctx& c, const void* src, void* dst) {
  if (c.lattice == 3) {
    if (c.precision == LBM_FP64) return dispatch_tile<3, false, double>(c, src, dst);
    return dispatch_tile<3, true, float>(c, src, dst);
  }
  if (c.precision == LBM_FP64) return dispatch_tile<2, false, double>(c, src, dst);
  return dispatch_tile<2, true, float>(c, src, dst);
}

hipError_t launch_init(const Ctx& c, const double* rho, const double* u, const double* T, void* dst) {
  const long long N = c.N;
  const dim3 grid((unsigned)((N + 255) / 256)), block(256);
  if (c.lattice == 3) {
    if (c.precision == LBM_FP64)
      hipLaunchKernelGGL((init_kernel<3, false, double>), grid, block, 0, c.stream, rho, u, T, (double*)dst, N, c.sp);
    else
      hipLaunchKernelGGL((init_kernel<3, true, float>), grid, block, 0, c.stream, rho, u, T, (float*)dst, N, c.sp);
  } else {
    if (c.precision == LBM_FP64)
      hipLaunchKernelGGL((init_kernel<2, false, double>), grid, block, 0, c.stream, rho, u, T, (double*)dst, N, c.sp);
    else
      hipLaunchKernelGGL((init_kernel<2, true, float>), grid, block, 0, c.stream, rho, u, T, (float*)dst, N, c.sp);
  }
  return hipGetLastError();
}

hipError_t launch_fields(const Ctx& c, const void* pops, double* fields) {
  const long long N = c.N;
  const dim3 grid((unsigned)((N + 255) / 256)), block(256);
  if (c.lattice == 3) {
    if (c.precision == LBM_FP64)
      hipLaunchKernelGGL((fields_kernel<3, false, double>), grid, block, 0, c.stream, (const double*)pops, fields, N,
                         c.sp);
    else
      hipLaunchKernelGGL((fields_kernel<3, true, float>), grid, block, 0, c.stream, (const float*)pops, fields, N,
                         c.sp);
  } else {
    if (c.precision == LBM_FP64)
      hipLaunchKernelGGL((fields_kernel<2, false, double>), grid, block, 0, c.stream, (const double*)pops, fields, N,
                         c.sp);
    else
      hipLaunchKernelGGL((fields_kernel<2, true, float>), grid, block, 0, c.stream, (const float*)pops, fields, N,
                         c.sp);
  }
  return hipGetLastError();
}

int diag_blocks(const Ctx& c) {
  const long long want = (c.N + 255) / 256;
  return (int)(want < 2048 ? want : 2048);
}

hipError_t launch_diag(const Ctx& c, const double* fields, double* partial, int nblocks, double* out) {
  if (c.lattice == 3)
    hipLaunchKernelGGL((diag_kernel<3>), dim3(nblocks), dim3(256), 0, c.stream, fields, partial, (long long)c.N, c.sp);
  else
    hipLaunchKernelGGL((diag_kernel<2>), dim3(nblocks), dim3(256), 0, c.stream, fields, partial, (long long)c.N, c.sp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((final_reduce_kernel<kNumDiag>), dim3(1), dim3(256), 0, c.stream, partial, nblocks, out);
  return hipGetLastError();
}

hipError_t launch_validate(const Ctx& c, const double* rho, const double* u, const double* T, double* partial,
                           int nblocks, double* out) {
  if (c.lattice == 3)
    hipLaunchKernelGGL((validate_kernel<3>), dim3(nblocks), dim3(256), 0, c.stream, rho, u, T, partial,
                       (long long)c.N);
  else
    hipLaunchKernelGGL((validate_kernel<2>), dim3(nblocks), dim3(256), 0, c.stream, rho, u, T, partial,
                       (long long)c.N);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((final_reduce_kernel<1>), dim3(1), dim3(256), 0, c.stream, partial, nblocks, out);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const long long n16 = (long long)(bytes / 16);
  long long blocks = (n16 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (const float4*)src, (float4*)dst, n16);
  return hipGetLastError();
}

}  // namespace lbm

namespace lbm {

hipError_t launch_pack(const Ctx& c, const void* pops, void* state) {
  const dim3 grid((unsigned)((c.N + 255) / 256)), block(256);
  if (c.precision == LBM_FP64)
    hipLaunchKernelGGL(pack_kernel<double>, grid, block, 0, c.stream, (const double*)pops, (double*)state,
                       (long long)c.N, 2 * c.Q, c.sp);
  else
    hipLaunchKernelGGL(pack_kernel<float>, grid, block, 0, c.stream, (const float*)pops, (float*)state,
                       (long long)c.N, 2 * c.Q, c.sp);
  return hipGetLastError();
}

hipError_t launch_unpack(const Ctx& c, const void* state, void* pops) {
  const dim3 grid((unsigned)((c.N + 255) / 256)), block(256);
  if (c.precision == LBM_FP64)
    hipLaunchKernelGGL(unpack_kernel<double>, grid, block, 0, c.stream, (const double*)state, (double*)pops,
                       (long long)c.N, 2 * c.Q, c.sp);
  else
    hipLaunchKernelGGL(unpack_kernel<float>, grid, block, 0, c.stream, (const float*)state, (float*)pops,
                       (long long)c.N, 2 * c.Q, c.sp);
  return hipGetLastError();
}

}  // namespace lbm
