// HIP kernels of liblbm.so (gfx950).
//
// Fused stream-and-collide (one launch per time step)
// ---------------------------------------------------
// Populations are stored plane-major: for every plane of the march axis (z
// for D3Q27, y for D2Q9) the Q velocity slots of that plane follow each
// other, each an in-plane array (x fastest) of (f_i, g_i) pairs:
//   buf[m * ms + i * 2 ps + 2 p + s],  p = in-plane node index,
//   s = 0 for f_i, 1 for g_i.
// f_i and g_i of a node stream from the same neighbour, so one 8-byte (FP32)
// or 16-byte (FP64) access moves both: half the memory instructions of
// separate arrays, and a wavefront touches a contiguous 512-byte (FP32) or
// 1-KB (FP64) run per slot.  A work-group that marches over a few planes
// touches a few MB of address space instead of 2Q arrays a whole field
// apart, which keeps the address translation caches warm.
// Streaming is done by pull: the thread of node x reads slot i from x - c_i
// (wrapped or clamped per axis) and writes the post-collision values at x.
//
// The anomaly correction needs, at node x, the post-streaming anomaly Qt_a of
// the neighbours x +- e_a of the same step.  A work-group owns a BX x BY tile
// of an in-plane slab and marches along the last axis (z for D3Q27, y for
// D2Q9) over a chunk of planes:
//   - each thread keeps its own node's post-streaming populations in
//     registers from the plane where they are loaded to the plane where they
//     are collided; the neighbours along the march axis are the same
//     thread's previous and next planes, held in registers.  The FP32 kernel
//     is software-pipelined two planes deep: while plane m collides, the
//     loads of plane m + 2 are in flight and plane m + 1 (loaded one
//     iteration earlier) supplies the anomaly along the march axis;
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

// Debug build switch (liblbm_poison.so): fill the step kernel's LDS anomaly
// ring with NaN at the start and before every plane refills its half, so
// that a value read without having been written for the current plane shows
// up as NaN in the results instead of a stale neighbour value.
#ifndef LBM_POISON_LDS
#define LBM_POISON_LDS 0
#endif

namespace lbm {

__device__ inline int fix_coord(int k, int n, int bc) {
  if (bc == LBM_BC_PERIODIC) {
    k %= n;
    return k < 0 ? k + n : k;
  }
  return k < 0 ? 0 : (k > n - 1 ? n - 1 : k);
}

// fix_coord for -n <= k < 3n without a division (march-plane indices).
__device__ inline int fix_near(int k, int n, int bc) {
  if (bc == LBM_BC_PERIODIC) {
    k = k < 0 ? k + n : k;
    k = k >= n ? k - n : k;
    return k >= n ? k - n : k;
  }
  return k < 0 ? 0 : (k > n - 1 ? n - 1 : k);
}

// Element offset of population i (f_i for i < Q, g_{i-Q} for i >= Q) of
// node n (node = x + nx*(y + ny*z)).
__device__ inline long long pop_offset(const StepParams& p, int Q, int i, long long n) {
  const long long m = n / p.plane;
  const long long q = n - m * p.plane;
  const int slot = i < Q ? i : i - Q;
  return m * p.ms + (q >> 6) * p.blk + (long long)slot * p.sl + 2 * (q & 63) + (i < Q ? 0 : 1);
}

// Byte offset of the (f, g) pair of slot 0 of in-plane node q within its
// march plane.
template <typename S>
__device__ inline unsigned inplane_bytes(const StepParams& p, int q) {
  return (unsigned)(((unsigned long long)(q >> 6) * (unsigned long long)p.blk + 2u * (unsigned)(q & 63)) * sizeof(S));
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
  k.cv1 = p.cv1;
  k.cv2 = p.cv2;
  k.U0 = p.U0;
  k.caloric = p.caloric;
  k.Pr = p.Pr;
  k.mu0 = p.mu0;
  k.visc_exp = p.visc_exp;
  k.inv_Tref = p.inv_Tref;
  for (int a = 0; a < 3; ++a) {
    k.u0[a] = p.u0[a];
    k.P0[a] = p.P0[a];
    k.u0f[a] = p.u0f[a];
    k.P0f[a] = p.P0f[a];
    for (int c = 0; c < 3; ++c) {
      k.psi0[a][c] = p.psi0[a][c];
      k.b0[a][c] = p.b0[a][c];
      k.psi0f[a][c] = p.psi0f[a][c];
      k.b0f[a][c] = p.b0f[a][c];
    }
  }
  return k;
}

// Raw buffer access: a wave-uniform resource (base of one march plane), a
// per-lane 32-bit byte offset (the in-plane node) and a wave-uniform scalar
// offset (the population), so a load or store needs no per-lane address
// arithmetic.  Offsets past the resource's size read 0 and drop writes.
constexpr int kBufferFlags = 0x00020000;  // raw 32-bit data format (gfx9 family)
// Cache policy of the step kernel's stores: default.  (Non-temporal stores
// measured 5% slower in this kernel on gfx950.)
constexpr int kStorePolicy = 0;

__device__ inline __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, long long bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufferFlags);
}

// One (f_i, g_i) pair per access.
template <typename S>
struct Buf;
template <>
struct Buf<float> {
  typedef float pair_t __attribute__((ext_vector_type(2)));
  static __device__ inline pair_t load(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    return __builtin_bit_cast(pair_t, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
  }
  static __device__ inline void store(pair_t v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, vo, so, kStorePolicy);
  }
};
template <>
struct Buf<double> {
  typedef double pair_t __attribute__((ext_vector_type(2)));
  static __device__ inline pair_t load(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    return __builtin_bit_cast(pair_t, __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0));
  }
  static __device__ inline void store(pair_t v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V, v), r, vo, so, kStorePolicy);
  }
};

// Pull-load the 2Q populations arriving at a node.  rs[k] is the resource of
// march plane (m + k - 1) after wrap/clamp; lo[j] is the byte offset inside a
// plane of the in-plane source (y + j/3 - 1, x + j%3 - 1).  Slot i of the
// source x - c_i sits at scalar offset i * slot_bytes of plane 1 - c_m.
template <int D, typename S, typename R>
__device__ inline void pull(const __amdgpu_buffer_rsrc_t* rs, unsigned slot_bytes, const unsigned* lo, R* f, R* g) {
  constexpr int Q = lat_q(D);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = vx(i);
    const int cy = (D == 3) ? vy(i) : 0;
    const int cm = (D == 3) ? vz(i) : vy(i);
    const unsigned o = lo[(1 - cy) * 3 + (1 - cx)];
    const auto v = Buf<S>::load(rs[1 - cm], o, (unsigned)i * slot_bytes);
    f[i] = (R)v.x;
    g[i] = (R)v.y;
  }
}

// Density, velocity and temperature of a node from its pulled populations,
// loaded and summed in batches of nine velocities so that few registers hold
// loaded values at a time (used for the halo node where registers are short).
template <int D, typename S, typename R>
__device__ inline NodeMoments<R> pulled_moments_batched(const __amdgpu_buffer_rsrc_t* rs, unsigned slot_bytes,
                                                        const unsigned* lo, const NodeConsts& k) {
  constexpr int Q = lat_q(D);
  double s0 = 0, j[3] = {0, 0, 0}, se = 0;
#pragma unroll
  for (int b = 0; b < Q; b += 9) {
    R f[9], g[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const int i = b + q;
      const int cx = vx(i);
      const int cy = (D == 3) ? vy(i) : 0;
      const int cm = (D == 3) ? vz(i) : vy(i);
      const auto v = Buf<S>::load(rs[1 - cm], lo[(1 - cy) * 3 + (1 - cx)], (unsigned)i * slot_bytes);
      f[q] = (R)v.x;
      g[q] = (R)v.y;
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const int i = b + q;
      const int cx = vx(i), cy = vy(i), cz = (D == 3) ? vz(i) : 0;
      s0 += f[q];
      se += g[q];
      if (cx) j[0] += cx > 0 ? f[q] : -f[q];
      if (cy) j[1] += cy > 0 ? f[q] : -f[q];
      if (cz) j[2] += cz > 0 ? f[q] : -f[q];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  NodeMoments<R> m;
  velocity_temperature<D, R>(m, s0, j, se, k);
  return m;
}

// Stand-ins for the node arithmetic in the access-pattern reference kernel
// (PAT): each keeps the values it is given live at the cost of about one
// addition per value, so that the kernel loads and stores exactly what a
// step does and computes nothing else.
template <int D, typename R>
__device__ inline NodeMoments<R> pattern_moments(const R* f, const R* g) {
  NodeMoments<R> m{};
#pragma unroll
  for (int a = 0; a < 3; ++a) m.u[a] = f[a] + g[a];
  return m;
}

// All 2Q values (the halo node and the plane before a chunk, where a step
// forms the conserved sums).
template <int D, typename R>
__device__ inline NodeMoments<R> pattern_all(const R* f, const R* g) {
  constexpr int Q = lat_q(D);
  R acc = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) acc += f[i] + g[i];
  NodeMoments<R> m{};
  m.u[0] = m.u[1] = m.u[2] = acc;
  return m;
}

template <int D, typename S, typename R>
__device__ inline NodeMoments<R> pattern_pulled(const __amdgpu_buffer_rsrc_t* rs, unsigned slot_bytes,
                                                const unsigned* lo) {
  constexpr int Q = lat_q(D);
  R acc = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = vx(i);
    const int cy = (D == 3) ? vy(i) : 0;
    const int cm = (D == 3) ? vz(i) : vy(i);
    const auto v = Buf<S>::load(rs[1 - cm], lo[(1 - cy) * 3 + (1 - cx)], (unsigned)i * slot_bytes);
    acc += (R)v.x + (R)v.y;
  }
  NodeMoments<R> m{};
  m.u[0] = m.u[1] = m.u[2] = acc;
  return m;
}

// One work-group's share of a step: tile lb (x fastest, then y, then the
// march chunk) of the box described by p.  CAL: the general caloric law
// (p.caloric must equal CAL); with CAL false the constant-C_v arithmetic is
// all the kernel contains.
// PAT: the access-pattern reference (same loads, stores, LDS exchange and
// barriers, no collision: the streamed populations are stored).
template <int D, bool DEV, typename S, int BX, int BY, bool CAL = false, bool PAT = false>
__device__ __forceinline__ void step_tile(const S* __restrict__ src, S* __restrict__ dst, const StepParams& p, int lb) {
  using R = typename StoreOf<S>::R;
  constexpr int Q = lat_q(D);
  constexpr int NHALO = (D == 3) ? 2 * BX + 2 * BY : 2;
  static_assert(BX * BY >= NHALO, "tile too small for its halo");
  static_assert(D == 3 || BY == 1, "D2Q9 tiles are one row");
  __shared__ R lq0[2][BY][BX + 2];                    // anomaly along in-plane axis 0 (x)
  __shared__ R lq1[2][(D == 3) ? BY + 2 : 1][BX];     // anomaly along in-plane axis 1 (y, D3Q27 only)
  // half b of the ring set to NaN by the whole work-group (debug build only;
  // the caller separates it from the next reads or writes by a barrier)
  auto poison = [&](int b) {
    constexpr int N0 = BY * (BX + 2), N1 = ((D == 3) ? BY + 2 : 1) * BX;
    const R nan = (R)__builtin_nan("");
    for (int e = threadIdx.x; e < N0; e += BX * BY) (&lq0[b][0][0])[e] = nan;
    for (int e = threadIdx.x; e < N1; e += BX * BY) (&lq1[b][0][0])[e] = nan;
  };
  if constexpr (LBM_POISON_LDS) {
    poison(0);
    poison(1);
    __syncthreads();
  }

  NodeConsts k = node_consts(p);
  k.caloric = CAL ? 1 : 0;
  if constexpr (!CAL) k.U0 = k.Cv * k.T0;  // the same value, formed from constants already held

  const int tx = lb % p.tiles_x;
  const int rest = lb / p.tiles_x;
  const int ty = (D == 3) ? rest % p.tiles_y : 0;
  const int ck = (D == 3) ? rest / p.tiles_y : rest;

  const int n0 = p.nx;
  const int n1 = (D == 3) ? p.ny : 1;
  const int nm = (D == 3) ? p.nz : p.ny;
  const int bc0 = p.bc[0], bc1 = p.bc[1], bcm = (D == 3) ? p.bc[2] : p.bc[1];
  const long long sm = p.ms;  // march-plane stride

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

  // FP32 with up to 256 threads per group: two planes in flight (see the
  // header), in up to 512 registers at one wavefront per SIMD.  FP64 needs
  // twice the registers per population, and 512-thread groups have half the
  // registers per thread: one plane in flight.
  // The pattern reference holds no arithmetic state, so it keeps two planes
  // in flight for every shape: the best latency hiding the access pattern
  // allows.
  constexpr bool PF2 = PAT || (DEV && BX * BY <= 256);
  // One plane in flight in a 512-thread group (two wavefronts per SIMD, both
  // of this group): the next core loads are issued before the barrier that
  // ends a plane, so their latency overlaps the wait for the wavefronts that
  // pull halo nodes.  At one wavefront per SIMD (256 threads) issuing them at
  // the top of the plane measured faster.
  constexpr bool EARLY = !PF2 && BX * BY > 256;
  const unsigned slot_bytes = (unsigned)(p.sl * (long long)sizeof(S));
  const long long plane_bytes = sm * (long long)sizeof(S);
  // byte offsets of the 9 in-plane sources of the core and of the halo node
  unsigned clo[9], hlo[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    clo[j] = inplane_bytes<S>(p, coy[j / 3] + cox[j % 3]);
    hlo[j] = inplane_bytes<S>(p, hoy[j / 3] + hox[j % 3]);
  }
  auto march_planes = [&](int m, __amdgpu_buffer_rsrc_t* rs) {
    const int mn = fix_near(m, nm, bcm);  // m0 - 1 <= m <= m1 + 1
#pragma unroll
    for (int j = 0; j < 3; ++j) rs[j] = plane_rsrc(src + (long long)fix_near(mn + j - 1, nm, bcm) * sm, plane_bytes);
  };
  // Node arithmetic (or its stand-ins in the pattern reference).
  auto anom = [&](const NodeMoments<R>& mm, int a) -> R {
    if constexpr (PAT) return mm.u[a];
    else return anomaly(mm, a, k);
  };
  auto moments = [&](const R* f, const R* g) -> NodeMoments<R> {
    if constexpr (PAT) return pattern_moments<D, R>(f, g);
    else return node_moments<D, R>(f, g, k);
  };
  auto moments_light = [&](const R* f, const R* g) -> NodeMoments<R> {
    if constexpr (PAT) return pattern_all<D, R>(f, g);
    else if constexpr (DEV) return node_moments_light<D>(f, g, k);
    else return node_moments<D, R>(f, g, k);
  };
  // The halo node's anomaly into LDS buffer buf.
  auto halo_store = [&](const NodeMoments<R>& mm, int buf) {
    if (D == 3) {
      if (hslot == 0) lq1[buf][0][t] = anom(mm, 1);
      else if (hslot == 1) lq1[buf][BY + 1][t - BX] = anom(mm, 1);
      else if (hslot == 2) lq0[buf][t - 2 * BX][0] = anom(mm, 0);
      else lq0[buf][t - 2 * BX - BY][BX + 1] = anom(mm, 0);
    } else {
      lq0[buf][0][hslot == 2 ? 0 : BX + 1] = anom(mm, 0);
    }
  };
  // ... from populations already in registers (FP32 only) ...
  auto halo_finish = [&](const R* f, const R* g, int buf) {
    if constexpr (DEV || PAT) {
      if (has_halo) halo_store(moments_light(f, g), buf);
    }
  };
  // ... or loaded now, in batches.
  auto halo_direct = [&](const __amdgpu_buffer_rsrc_t* rs, int buf) {
    if (has_halo) {
      if constexpr (PAT) halo_store(pattern_pulled<D, S, R>(rs, slot_bytes, hlo), buf);
      else halo_store(pulled_moments_batched<D, S, R>(rs, slot_bytes, hlo, k), buf);
    }
  };
  // Own node's in-plane anomalies into LDS buffer buf.
  auto core_publish = [&](const NodeMoments<R>& mm, int buf) {
    lq0[buf][ly][lx + 1] = anom(mm, 0);
    if (D == 3) lq1[buf][ly + 1][lx] = anom(mm, 1);
  };

  R qm_prev, qm_cur, qm_next;  // anomaly along the march axis at m - 1, m, m + 1
  R hf[Q], hg[Q];              // halo node populations (in flight for the next plane)
  R f0[Q], g0[Q], f1[Q], g1[Q], f2[Q], g2[Q];
  NodeMoments<R> mo0, mo1, mo2;
  // prologue: anomaly along the march axis at plane m0 - 1 (core only)
  {
    __amdgpu_buffer_rsrc_t rs[3];
    march_planes(m0 - 1, rs);
    pull<D, S, R>(rs, slot_bytes, clo, f0, g0);
    const NodeMoments<R> mm = moments_light(f0, g0);
    qm_prev = anom(mm, D - 1);
  }
  // plane m0: core populations stay in registers, in-plane anomaly to LDS
  {
    __amdgpu_buffer_rsrc_t rs[3];
    march_planes(m0, rs);
    pull<D, S, R>(rs, slot_bytes, clo, f0, g0);
    mo0 = moments(f0, g0);
    qm_cur = anom(mo0, D - 1);
    core_publish(mo0, 0);
    halo_direct(rs, 0);
  }
  {
    __amdgpu_buffer_rsrc_t rs[3];
    march_planes(m0 + 1, rs);
    if (PF2 || EARLY) pull<D, S, R>(rs, slot_bytes, clo, f1, g1);
    if (PF2 && has_halo) pull<D, S, R>(rs, slot_bytes, hlo, hf, hg);
  }
  __syncthreads();

  // One plane: collide plane m (fa, ga, ma) and finish plane m + 1 (fb, gb,
  // mb).  PF2: plane m + 1's loads were issued one plane earlier, and the
  // loads of plane m + 2 (core and halo) go into (fc, gc) before the
  // collision; the three register sets rotate through a 3-way unrolled loop.
  // One plane in flight: plane m + 1 moves into (fa, ga) once plane m is
  // stored; its core loads were issued at the end of the previous plane
  // (EARLY) or at the top of this one.
  auto plane = [&](int m, R* fa, R* ga, NodeMoments<R>& ma, R* fb, R* gb, NodeMoments<R>& mb, R* fc, R* gc) {
    const int cb = (m - m0) & 1, nb = cb ^ 1;
    const bool more = m + 1 < m1;  // plane m + 1 collides in this chunk
    if constexpr (LBM_POISON_LDS) {
      // half nb was last read by plane m - 1, which ended with a barrier
      poison(nb);
      __syncthreads();
    }
    if (PF2) {
      __amdgpu_buffer_rsrc_t rs[3];
      march_planes(more ? m + 2 : m + 1, rs);
      if (more) pull<D, S, R>(rs, slot_bytes, clo, fc, gc);
      mb = moments(fb, gb);
      qm_next = anom(mb, D - 1);
      core_publish(mb, nb);
      halo_finish(hf, hg, nb);
      if (more && has_halo) pull<D, S, R>(rs, slot_bytes, hlo, hf, hg);
    } else {
      // one plane in flight; the halo node's populations are loaded in
      // batches, so only one batch of them is live beside the two core sets
      __amdgpu_buffer_rsrc_t rs[3];
      march_planes(m + 1, rs);
      if constexpr (EARLY) {
        // the halo first: its loads then overlap the latency of plane
        // m + 1's core loads, issued before the barrier (1.3 % faster than
        // pulling it after the core moments)
        halo_direct(rs, nb);
        mb = moments(fb, gb);
        qm_next = anom(mb, D - 1);
        core_publish(mb, nb);
      } else {
        pull<D, S, R>(rs, slot_bytes, clo, fb, gb);
        mb = moments(fb, gb);
        qm_next = anom(mb, D - 1);
        core_publish(mb, nb);
        halo_direct(rs, nb);
      }
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
    if constexpr (PAT) fa[0] += (dd[0] + dd[1]) + dd[2];
    else collide<D, R, DEV>(fa, ga, ma, dd, k);
    if (active) {
      const __amdgpu_buffer_rsrc_t rd = plane_rsrc(dst + (long long)m * sm, plane_bytes);
      const unsigned o = inplane_bytes<S>(p, cnode);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        typename Buf<S>::pair_t v;
        v.x = (S)fa[i];
        v.y = (S)ga[i];
        Buf<S>::store(v, rd, o, (unsigned)i * slot_bytes);
      }
    }
    if (!PF2) {
      // plane m + 1 becomes the next collision set (EARLY: plane m + 2's
      // loads go into the freed set now)
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        fa[i] = fb[i];
        ga[i] = gb[i];
      }
      ma = mb;
      if (EARLY && more) {
        __amdgpu_buffer_rsrc_t rs[3];
        march_planes(m + 2, rs);
        pull<D, S, R>(rs, slot_bytes, clo, fb, gb);
      }
    }
    __syncthreads();
    qm_prev = qm_cur;
    qm_cur = qm_next;
  };

  if (PF2) {
    // sets: plane m in 0, m + 1 in 1, m + 2 loads into 2; then rotate
    for (int m = m0; m < m1; m += 3) {
      plane(m, f0, g0, mo0, f1, g1, mo1, f2, g2);
      if (m + 1 >= m1) break;
      plane(m + 1, f1, g1, mo1, f2, g2, mo2, f0, g0);
      if (m + 2 >= m1) break;
      plane(m + 2, f2, g2, mo2, f0, g0, mo0, f1, g1);
    }
  } else {
    // plane m in set 0, plane m + 1 in flight in set 1
    for (int m = m0; m < m1; ++m) plane(m, f0, g0, mo0, f1, g1, mo1, f2, g2);
  }
}

// XCD-aware logical block: consecutive hardware block ids go round the eight
// XCDs, so logical blocks are renumbered such that each XCD runs one
// contiguous range (neighbouring tiles then share an L2).
__device__ inline int xcd_logical_block(int b, int nblocks) {
  const int q8 = nblocks >> 3, r8 = nblocks & 7, xcd = b & 7;
  return xcd * q8 + min(xcd, r8) + (b >> 3);
}

template <int D, bool DEV, typename S, int BX, int BY, bool CAL = false>
__global__ void __launch_bounds__(BX* BY) step_kernel(const S* __restrict__ src, S* __restrict__ dst,
                                                      const StepParams p) {
  step_tile<D, DEV, S, BX, BY, CAL>(src, dst, p, xcd_logical_block(blockIdx.x, p.nblocks));
}

// The access-pattern reference of step_kernel (see step_tile).
template <int D, bool DEV, typename S, int BX, int BY>
__global__ void __launch_bounds__(BX* BY) pattern_kernel(const S* __restrict__ src, S* __restrict__ dst,
                                                         const StepParams p) {
  step_tile<D, DEV, S, BX, BY, false, true>(src, dst, p, xcd_logical_block(blockIdx.x, p.nblocks));
}

// Several boxes in one launch: logical block g belongs to the last box whose
// first block is <= g; that box's current buffer (cur ^ flip) is the source.
template <int D, bool DEV, typename S, int BX, int BY>
__global__ void __launch_bounds__(BX* BY) batch_step_kernel(const BoxEntry* __restrict__ table, int nboxes,
                                                            int total_blocks, int flip) {
  const int g = xcd_logical_block(blockIdx.x, total_blocks);
  int lo = 0, hi = nboxes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (table[mid].block_start <= g) lo = mid;
    else hi = mid - 1;
  }
  const BoxEntry& e = table[lo];
  const int par = e.cur ^ flip;
  step_tile<D, DEV, S, BX, BY>(static_cast<const S*>(e.buf[par]), static_cast<S*>(e.buf[par ^ 1]), e.p,
                               g - e.block_start);
}

// The same step with a fixed grid (a few work-groups per compute unit, sized
// by occupancy): each XCD owns one contiguous eighth of the logical tiles
// (neighbouring tiles share its L2) and its work-groups take that range's
// tiles in turn, tile rank, rank + (work-groups per XCD), ...  Every
// work-group leaves the loop when its range is done; no work-group waits
// for another.  gridDim.x is a multiple of 8.
template <int D, bool DEV, typename S, int BX, int BY>
__global__ void __launch_bounds__(BX* BY) batch_persistent_kernel(const BoxEntry* __restrict__ table, int nboxes,
                                                                  int total_blocks, int flip) {
  const int per_xcd = gridDim.x >> 3, xcd = blockIdx.x & 7, rank = blockIdx.x >> 3;
  const int lo = (int)((long long)total_blocks * xcd / 8), hi = (int)((long long)total_blocks * (xcd + 1) / 8);
  for (int g = lo + rank; g < hi; g += per_xcd) {
    int a = 0, z = nboxes - 1;
    while (a < z) {
      const int mid = (a + z + 1) >> 1;
      if (table[mid].block_start <= g) a = mid;
      else z = mid - 1;
    }
    const BoxEntry& e = table[a];
    const int par = e.cur ^ flip;
    step_tile<D, DEV, S, BX, BY>(static_cast<const S*>(e.buf[par]), static_cast<S*>(e.buf[par ^ 1]), e.p,
                                 g - e.block_start);
  }
}

// After an odd number of batched steps every box's current buffer changes.
__global__ void __launch_bounds__(64) toggle_cur_kernel(BoxEntry* __restrict__ table, int nboxes) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nboxes) table[i].cur ^= 1;
}

// ---------------------------------------------------------------------------
// Initialisation: f = f^eq, g = g^eq (minus the reference state when DEV).
// The equilibria are evaluated in FP64 for either storage, so FP32 storage
// holds each deviation rounded once.
// ---------------------------------------------------------------------------

template <int D, bool DEV, typename S>
__global__ void __launch_bounds__(256) init_kernel(const double* __restrict__ rho, const double* __restrict__ u,
                                                   const double* __restrict__ T, S* __restrict__ dst, long long N,
                                                   const StepParams p) {
  using R = double;
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
  for (int a = 0; a < 3; ++a) {
    const double ua = a < D ? u[a * N + n] : 0.0;
    m.u[a] = (R)ua;
    m.du[a] = (R)(ua - p.u0[a]);
  }
  m.omega = m.omega1 = (R)1;  // unused by the equilibria
  m.corr = (R)0;                // multiplies d = 0
  R d[3] = {0, 0, 0};
  R fe[Q], ge[Q];
  equilibria<D, R, DEV>(m, d, k, fe, ge);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    dst[pop_offset(p, Q, i, n)] = (S)fe[i];
    dst[pop_offset(p, Q, i + Q, n)] = (S)ge[i];
  }
}

// ---------------------------------------------------------------------------
// Moments of the stored populations (no streaming), FP64 fields
// fields: rho, ux, uy, uz, T, rhoE (each N)
// ---------------------------------------------------------------------------

// Sums of the stored values of node n: s0 = sum f, j = sum c f and, when se
// is not NULL, *se = sum g (in population order).
template <int D, typename S>
__device__ inline void stored_sums(const S* __restrict__ pops, const StepParams& p, long long n, double& s0,
                                   double* j, double* se) {
  constexpr int Q = lat_q(D);
  double jx = 0, jy = 0, jz = 0, e = 0;
  s0 = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double v = (double)pops[pop_offset(p, Q, i, n)];
    s0 += v;
    if (se) e += (double)pops[pop_offset(p, Q, i + Q, n)];
    const int cx = vx(i), cy = vy(i), cz = (D == 3) ? vz(i) : 0;
    if (cx) jx += cx > 0 ? v : -v;
    if (cy) jy += cy > 0 ? v : -v;
    if (cz) jz += cz > 0 ? v : -v;
  }
  j[0] = jx;
  j[1] = jy;
  j[2] = jz;
  if (se) *se = e;
}

// rho and u of node n from its stored populations (FP64).
template <int D, typename S>
__device__ inline double stored_velocity(const S* __restrict__ pops, const StepParams& p, long long n, double* u) {
  double s0, j[3];
  stored_sums<D, S>(pops, p, n, s0, j, nullptr);
  const double rho = p.rho0 + s0;
  u[0] = (p.j0[0] + j[0]) / rho;
  u[1] = (p.j0[1] + j[1]) / rho;
  u[2] = (D == 3) ? (p.j0[2] + j[2]) / rho : 0.0;
  return rho;
}

// rho, u, T and rho E of node n from its stored populations (FP64; Eqs.
// (3)-(7) without streaming).
template <int D, typename S>
__device__ inline void stored_fields(const S* __restrict__ pops, const StepParams& p, long long n, double& rho,
                                     double* u, double& T, double& rhoE) {
  double s0, j[3], se;
  stored_sums<D, S>(pops, p, n, s0, j, &se);
  rho = p.rho0 + s0;
  u[0] = (p.j0[0] + j[0]) / rho;
  u[1] = (p.j0[1] + j[1]) / rho;
  u[2] = (D == 3) ? (p.j0[2] + j[2]) / rho : 0.0;
  rhoE = p.rhoE0 + se;
  const double e = rhoE / rho - 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);  // U(T)
  T = p.caloric ? p.T0 + caloric_step(p.Cv, p.cv1, p.cv2, p.T0, e - p.U0) : e * p.inv_Cv;
}

template <int D, bool DEV, typename S>
__global__ void __launch_bounds__(256) fields_kernel(const S* __restrict__ pops, double* __restrict__ fields,
                                                     long long N, const StepParams p) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  double rho, u[3], T, rhoE;
  stored_fields<D, S>(pops, p, n, rho, u, T, rhoE);
  fields[n] = rho;
  fields[N + n] = u[0];
  fields[2 * N + n] = u[1];
  fields[3 * N + n] = u[2];
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

// Node indices of the six neighbours x+-1, y+-1, z+-1 of node n (wrap or
// clamp per axis): nb[0] = x+1, nb[1] = x-1, nb[2] = y+1, nb[3] = y-1,
// nb[4] = z+1, nb[5] = z-1.
__device__ inline void neighbours6(const StepParams& p, long long n, long long* nb) {
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int x = (int)(n % nx);
  const int y = (int)((n / nx) % ny);
  const int z = (int)(n / ((long long)nx * ny));
  auto idx = [&](int xx, int yy, int zz) { return xx + (long long)nx * (yy + (long long)ny * zz); };
  nb[0] = idx(fix_node_axis(x + 1, nx, p.bc[0]), y, z);
  nb[1] = idx(fix_node_axis(x - 1, nx, p.bc[0]), y, z);
  nb[2] = idx(x, fix_node_axis(y + 1, ny, p.bc[1]), z);
  nb[3] = idx(x, fix_node_axis(y - 1, ny, p.bc[1]), z);
  nb[4] = idx(x, y, fix_node_axis(z + 1, nz, p.bc[2]));
  nb[5] = idx(x, y, fix_node_axis(z - 1, nz, p.bc[2]));
}

// One node's terms of the 21 diagnostic sums (the totals of Eqs. (3)-(5)
// and the statistics of Sec. III.D), with central differences from the
// velocities vn[k] of the six neighbours (order of neighbours6).
template <int D>
__device__ inline void diag_accumulate(double (&acc)[kNumDiag], const StepParams& p, double rho, const double* u,
                                       double T, double rhoE, const double (*vn)[3]) {
  const double ux = u[0], uy = u[1], uz = u[2];
  // central differences d_b u_a
  const double dxux = 0.5 * (vn[0][0] - vn[1][0]);
  const double dyuy = 0.5 * (vn[2][1] - vn[3][1]);
  const double dzuz = (D == 3) ? 0.5 * (vn[4][2] - vn[5][2]) : 0.0;
  const double dxuy = 0.5 * (vn[0][1] - vn[1][1]);
  const double dyux = 0.5 * (vn[2][0] - vn[3][0]);
  double wx = 0.0, wy = 0.0;
  if (D == 3) {
    wx = 0.5 * (vn[2][2] - vn[3][2]) - 0.5 * (vn[4][1] - vn[5][1]);
    wy = 0.5 * (vn[4][0] - vn[5][0]) - 0.5 * (vn[0][2] - vn[1][2]);
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
  double gam = p.gamma;  // C_p / C_v at T (Mayer: C_p = C_v + 1)
  if (p.caloric) {
    const double cvT = caloric_cv(p.Cv, p.cv1, p.cv2, T);
    gam = (cvT + 1.0) / cvT;
  }
  acc[8] += sqrt(gam * T);
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

// Diagnostics from the field buffer F (rho, u_x, u_y, u_z, T, rho E planes).
template <int D>
__global__ void __launch_bounds__(256) diag_kernel(const double* __restrict__ F, double* __restrict__ partial,
                                                   long long N, const StepParams p) {
  double acc[kNumDiag];
#pragma unroll
  for (int j = 0; j < kNumDiag; ++j) acc[j] = 0.0;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
    long long nb[6];
    neighbours6(p, n, nb);
    double vn[6][3];
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
      for (int a = 0; a < 3; ++a) vn[k][a] = F[(long long)(1 + a) * N + nb[k]];
    const double u[3] = {F[N + n], F[2 * N + n], F[3 * N + n]};
    diag_accumulate<D>(acc, p, F[n], u, F[4 * N + n], F[5 * N + n], vn);
  }
  block_reduce_store<kNumDiag>(acc, partial + (long long)blockIdx.x * kNumDiag);
}

// The same sums straight from the stored populations: every node forms its
// own fields and its neighbours' velocities from the populations with the
// arithmetic of fields_kernel, so the terms, and with the same grid the
// sums, are those of fields_kernel + diag_kernel; no field buffer is needed.
template <int D, typename S>
__global__ void __launch_bounds__(256) diag_direct_kernel(const S* __restrict__ pops, double* __restrict__ partial,
                                                          long long N, const StepParams p) {
  double acc[kNumDiag];
#pragma unroll
  for (int j = 0; j < kNumDiag; ++j) acc[j] = 0.0;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
    long long nb[6];
    neighbours6(p, n, nb);
    double vn[6][3];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      if (D == 2 && k >= 4) {  // no z neighbours: the (unused) z differences see the node itself
        vn[k][0] = vn[k][1] = vn[k][2] = 0.0;
        continue;
      }
      stored_velocity<D, S>(pops, p, nb[k], vn[k]);
    }
    double rho, u[3], T, rhoE;
    stored_fields<D, S>(pops, p, n, rho, u, T, rhoE);
    diag_accumulate<D>(acc, p, rho, u, T, rhoE, vn);
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
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n16) dst[i] = src[i];
}

template <typename S>
__global__ void __launch_bounds__(256) pack_kernel(const S* __restrict__ pops, S* __restrict__ state, long long N,
                                                   int nq, const StepParams p) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  for (int i = 0; i < nq; ++i) state[(long long)i * N + n] = pops[pop_offset(p, nq / 2, i, n)];
}

template <typename S>
__global__ void __launch_bounds__(256) unpack_kernel(const S* __restrict__ state, S* __restrict__ pops, long long N,
                                                     int nq, const StepParams p) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  for (int i = 0; i < nq; ++i) pops[pop_offset(p, nq / 2, i, n)] = state[(long long)i * N + n];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

template <int D, bool DEV, typename S, int BX, int BY, bool CAL = false>
static hipError_t launch_step_t(const Ctx& c, const void* src, void* dst) {
  hipLaunchKernelGGL((step_kernel<D, DEV, S, BX, BY, CAL>), dim3(c.sp.nblocks), dim3(BX * BY), 0, c.stream,
                     static_cast<const S*>(src), static_cast<S*>(dst), c.sp);
  return hipGetLastError();
}

// Estimated time of a 3-D launch, in units of one 64 x 4 tile plane.  A
// work-group marches `chunk` planes of one tile column and occupies a whole
// CU (one wavefront per SIMD for the 256-thread shapes, two for 64 x 8), so
// the launch runs in rounds of 256 work-groups.  Each chunk pays a prologue
// (the planes next to it are loaded and their moments computed before its
// first collision) worth about 8 planes in the measured chunk sweeps.  w is
// the time of one tile plane of the shape relative to 64 x 4: 32 x 8 moves
// the same nodes a little slower (1.02), 64 x 8 moves twice the nodes with
// two wavefronts per SIMD hiding more latency (1.8).
static double march_cost(const int64_t n[3], int bx, int by, int64_t chunk, double w, double pro) {
  const int64_t tiles = ((n[0] + bx - 1) / bx) * ((n[1] + by - 1) / by);
  const int64_t blocks = tiles * ((n[2] + chunk - 1) / chunk);
  return (double)((blocks + 255) / 256) * ((double)chunk + pro) * w;
}

// Per-plane cost w and chunk prologue pro (in planes) of a 3-D launch shape,
// fitted to tile and chunk sweeps: 64 x 4 (1, 8 planes), 32 x 8 (1.02, 8)
// and the 512-thread 64 x 8 (1.82, 4.45; its next plane's loads are issued
// before the per-plane barrier, which shortens its prologue: fitted to
// 256^3 in 128-plane chunks and a 256 x 256 x 32 slab in 16-plane chunks).
static double shape_prologue(int bx, int by) { return (bx == 64 && by == 8) ? 4.45 : 8.0; }

// The power-of-two chunk of 4 to 256 planes, or the whole march axis, with
// the lowest march_cost for one 3-D launch shape.  Chunks stay powers of
// two: at 80^3 and 96^3, 8- and 16-plane chunks ran up to 45% faster than
// 6-, 12- or 24-plane ones.
static int64_t best_chunk3(const int64_t n[3], int bx, int by, double w, double* cost) {
  int64_t best = 1;
  double best_cost = -1.0;
  const double pro = shape_prologue(bx, by);
  for (int64_t chunk = 4;; chunk *= 2) {
    const int64_t c = chunk < n[2] ? chunk : n[2];
    const double k = march_cost(n, bx, by, c, w, pro);
    if (best_cost < 0.0 || k < best_cost) {
      best_cost = k;
      best = c;
    }
    if (chunk >= n[2] || chunk >= 256) break;
  }
  if (cost) *cost = best_cost;
  return best;
}

int default_chunk(int D, const int64_t n[3], int bx, int by) {
  if (D == 3) return (int)best_chunk3(n, bx, by, 1.0, nullptr);
  // D2Q9: chunks short enough for about 2^17 threads in flight (1024
  // work-groups of 128; the whole 2-D field is small), between 4 and 32 rows.
  const int64_t tiles = (n[0] + bx - 1) / bx;
  int64_t chunk = n[1] * tiles * bx / (1024 * 128);
  chunk = chunk < 4 ? 4 : (chunk > 32 ? 32 : chunk);
  return (int)(chunk < n[1] ? chunk : n[1]);
}

// Default launch shape and march chunk (32 x 16 tiles, the 512-thread shape
// with the smallest halo ring, measured 10% slower than 64 x 8 at 256^3 FP32
// and are not compiled).  D3Q27: the compiled shape with the
// lowest march_cost at its best chunk — 64 x 4, 32 x 8 and, for FP32
// storage, 64 x 8 (the only 512-thread shape that fits 256 registers
// without spilling); the caloric variant is compiled for 64 x 4 only.  On
// one MI355X this picks 64 x 4 with 4-plane chunks at 64^3 (2.1x the
// throughput of 16-plane chunks), 32 x 8 / 16 at 96^3, 64 x 8 / 16 at 128^3
// (3.6% faster than 64 x 4 / 32), 64 x 8 / 64 at 192^3, 64 x 8 / 128 at
// 256^3 (9% faster than 64 x 4 / 256 there) and 64 x 8 / 16 for a
// 256 x 256 x 32 slab (8% faster than 64 x 4 / 32).  D2Q9: rows of 128, or of 256 from 1024 nodes per row
// (FP32: 9% faster at 4096^2, even at 1024^2 and 2048^2; FP64 at 1024^2: 4%
// faster).
Tile default_tile(int D, int precision, const int64_t n[3], bool caloric) {
  if (D == 3) {
    struct Shape { int bx, by; double w; };
    const Shape shapes[3] = {{64, 4, 1.0}, {32, 8, 1.02}, {64, 8, 1.82}};
    const int nshapes = caloric ? 1 : (precision == LBM_FP32_DEV ? 3 : 2);
    Tile best{64, 4, 1};
    double best_cost = -1.0;
    for (int s = 0; s < nshapes; ++s) {
      double k = 0.0;
      const int64_t c = best_chunk3(n, shapes[s].bx, shapes[s].by, shapes[s].w, &k);
      if (best_cost < 0.0 || k < best_cost) {
        best_cost = k;
        best = Tile{shapes[s].bx, shapes[s].by, (int)c};
      }
    }
    return best;
  }
  const int bx = (!caloric && n[0] >= 1024) ? 256 : 128;
  return Tile{bx, 1, default_chunk(D, n, bx, 1)};
}

// The 512-thread 64 x 8 shape exists for FP32 storage only: with FP64
// populations it does not fit the registers of two wavefronts per SIMD and
// spills, so it is not compiled for FP64.
bool tile_supported(int D, int precision, const Tile& t, bool caloric) {
  if (caloric) return D == 3 ? (t.bx == 64 && t.by == 4) : (t.bx == 128 && t.by == 1);
  if (D == 3)
    return (t.bx == 64 && t.by == 4) || (t.bx == 32 && t.by == 8) ||
           (t.bx == 64 && t.by == 8 && precision == LBM_FP32_DEV);
  return t.by == 1 && (t.bx == 64 || t.bx == 128 || t.bx == 256);
}

template <int D, bool DEV, typename S>
static hipError_t dispatch_tile(const Ctx& c, const void* src, void* dst) {
  const Tile& t = c.tile;
  if (c.sp.caloric) {  // the general caloric law: the default shape only
    if constexpr (D == 3) {
      if (t.bx == 64 && t.by == 4) return launch_step_t<D, DEV, S, 64, 4, true>(c, src, dst);
    } else {
      if (t.bx == 128) return launch_step_t<D, DEV, S, 128, 1, true>(c, src, dst);
    }
    return hipErrorInvalidValue;
  }
  if constexpr (D == 3) {
    if (t.bx == 64 && t.by == 4) return launch_step_t<D, DEV, S, 64, 4>(c, src, dst);
    if constexpr (DEV)
      if (t.bx == 64 && t.by == 8) return launch_step_t<D, DEV, S, 64, 8>(c, src, dst);
    if (t.bx == 32 && t.by == 8) return launch_step_t<D, DEV, S, 32, 8>(c, src, dst);
  } else {
    if (t.bx == 64) return launch_step_t<D, DEV, S, 64, 1>(c, src, dst);
    if (t.bx == 128) return launch_step_t<D, DEV, S, 128, 1>(c, src, dst);
    if (t.bx == 256) return launch_step_t<D, DEV, S, 256, 1>(c, src, dst);
  }
  return hipErrorInvalidValue;
}

template <int D, bool DEV, typename S, int BX, int BY>
static hipError_t launch_pattern_t(const Ctx& c, const void* src, void* dst) {
  hipLaunchKernelGGL((pattern_kernel<D, DEV, S, BX, BY>), dim3(c.sp.nblocks), dim3(BX * BY), 0, c.stream,
                     static_cast<const S*>(src), static_cast<S*>(dst), c.sp);
  return hipGetLastError();
}

template <int D, bool DEV, typename S>
static hipError_t dispatch_pattern(const Ctx& c, const void* src, void* dst) {
  const Tile& t = c.tile;
  if constexpr (D == 3) {
    if (t.bx == 64 && t.by == 4) return launch_pattern_t<D, DEV, S, 64, 4>(c, src, dst);
    if constexpr (DEV)
      if (t.bx == 64 && t.by == 8) return launch_pattern_t<D, DEV, S, 64, 8>(c, src, dst);
    if (t.bx == 32 && t.by == 8) return launch_pattern_t<D, DEV, S, 32, 8>(c, src, dst);
  } else {
    if (t.bx == 64) return launch_pattern_t<D, DEV, S, 64, 1>(c, src, dst);
    if (t.bx == 128) return launch_pattern_t<D, DEV, S, 128, 1>(c, src, dst);
    if (t.bx == 256) return launch_pattern_t<D, DEV, S, 256, 1>(c, src, dst);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_pattern(const Ctx& c, const void* src, void* dst) {
  if (c.lattice == 3) {
    if (c.precision == LBM_FP64) return dispatch_pattern<3, false, double>(c, src, dst);
    return dispatch_pattern<3, true, float>(c, src, dst);
  }
  if (c.precision == LBM_FP64) return dispatch_pattern<2, false, double>(c, src, dst);
  return dispatch_pattern<2, true, float>(c, src, dst);
}

hipError_t launch_step(const Ctx& c, const void* src, void* dst) {
  if (c.lattice == 3) {
    if (c.precision == LBM_FP64) return dispatch_tile<3, false, double>(c, src, dst);
    return dispatch_tile<3, true, float>(c, src, dst);
  }
  if (c.precision == LBM_FP64) return dispatch_tile<2, false, double>(c, src, dst);
  return dispatch_tile<2, true, float>(c, src, dst);
}

// Work-groups of the persistent batched launch: the occupancy of the kernel
// times the compute units, rounded down to a multiple of 8 (the XCDs).  0
// (one work-group per tile instead) when that covers every tile: rounding a
// grid near the tile count down would leave a few work-groups two tiles.
template <int D, bool DEV, typename S, int BX, int BY>
static hipError_t persistent_grid(const Batch& b, int* grid) {
  int per_cu = 0, cus = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_persistent_kernel<D, DEV, S, BX, BY>,
                                                              BX * BY, 0);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b.device);
  if (e != hipSuccess) return e;
  const int g = (per_cu * cus / 8) * 8;
  *grid = per_cu * cus < b.total_blocks && g >= 8 ? g : 0;
  return hipSuccess;
}

bool persistent_supported(const Tile& t) { return t.bx * t.by <= 256; }

template <int D, bool DEV, typename S, int BX, int BY>
static hipError_t launch_batch_t(const Batch& b, hipStream_t s, int flip) {
  // The looped tile body of a 512-work-item tile does not fit the register
  // file without a stack frame, so that form exists for tiles of at most 256
  // work-items only (the host refuses the combination).
  if constexpr (BX * BY <= 256) {
    if (b.persistent) {
      int grid = 0;
      const hipError_t e = persistent_grid<D, DEV, S, BX, BY>(b, &grid);
      if (e != hipSuccess) return e;
      if (grid > 0) {
        hipLaunchKernelGGL((batch_persistent_kernel<D, DEV, S, BX, BY>), dim3(grid), dim3(BX * BY), 0, s, b.table,
                           (int)b.boxes.size(), b.total_blocks, flip);
        return hipGetLastError();
      }
    }
  } else {
    if (b.persistent) return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL((batch_step_kernel<D, DEV, S, BX, BY>), dim3(b.total_blocks), dim3(BX * BY), 0, s, b.table,
                     (int)b.boxes.size(), b.total_blocks, flip);
  return hipGetLastError();
}

template <int D, bool DEV, typename S>
static hipError_t dispatch_batch(const Batch& b, hipStream_t s, int flip) {
  const Tile& t = b.tile;
  if constexpr (D == 3) {
    if (t.bx == 64 && t.by == 4) return launch_batch_t<D, DEV, S, 64, 4>(b, s, flip);
    if constexpr (DEV)
      if (t.bx == 64 && t.by == 8) return launch_batch_t<D, DEV, S, 64, 8>(b, s, flip);
    if (t.bx == 32 && t.by == 8) return launch_batch_t<D, DEV, S, 32, 8>(b, s, flip);
  } else {
    if (t.bx == 64) return launch_batch_t<D, DEV, S, 64, 1>(b, s, flip);
    if (t.bx == 128) return launch_batch_t<D, DEV, S, 128, 1>(b, s, flip);
    if (t.bx == 256) return launch_batch_t<D, DEV, S, 256, 1>(b, s, flip);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch_step(const Batch& b, hipStream_t s, int flip) {
  if (b.lattice == 3) {
    if (b.precision == LBM_FP64) return dispatch_batch<3, false, double>(b, s, flip);
    return dispatch_batch<3, true, float>(b, s, flip);
  }
  if (b.precision == LBM_FP64) return dispatch_batch<2, false, double>(b, s, flip);
  return dispatch_batch<2, true, float>(b, s, flip);
}

hipError_t launch_toggle(const Batch& b, hipStream_t s) {
  const int n = (int)b.boxes.size();
  hipLaunchKernelGGL(toggle_cur_kernel, dim3((n + 63) / 64), dim3(64), 0, s, b.table, n);
  return hipGetLastError();
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

// ---------------------------------------------------------------------------
// Field increments by re-equilibration, and the conservative box filter
// ---------------------------------------------------------------------------

// f_i += f^eq_i(new) - f^eq_i(old), g likewise (equilibria evaluated in FP64
// for either storage).  oldf, newf: rho, ux, uy, uz, T planes (N each).
template <int D, bool DEV, typename S>
__global__ void __launch_bounds__(256) fields_add_kernel(S* __restrict__ pops, const double* __restrict__ oldf,
                                                         const double* __restrict__ newf, long long N,
                                                         const StepParams p) {
  constexpr int Q = lat_q(D);
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const NodeConsts k = node_consts(p);
  double fo[Q], go[Q], fn[Q], gn[Q];
  const double d0[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    const double* F = w ? newf : oldf;
    NodeMoments<double> m;
    m.rho = F[n];
    m.drho = F[n] - p.rho0;
    m.T = F[4 * N + n];
    m.dT = F[4 * N + n] - p.T0;
    for (int a = 0; a < 3; ++a) {
      const double ua = a < D ? F[(1 + a) * N + n] : 0.0;
      m.u[a] = ua;
      m.du[a] = ua - p.u0[a];
    }
    m.omega = m.omega1 = 1.0;
    m.corr = 0.0;
    if (w) equilibria<D, double, DEV>(m, d0, k, fn, gn);
    else equilibria<D, double, DEV>(m, d0, k, fo, go);
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    S& fi = pops[pop_offset(p, Q, i, n)];
    S& gi = pops[pop_offset(p, Q, i + Q, n)];
    fi = (S)((double)fi + (fn[i] - fo[i]));
    gi = (S)((double)gi + (gn[i] - go[i]));
  }
}

// new = keep * old + d (rho, u planes, T); d: drho[N], du[D N], dT[N]; keep is
// 1 (increments) or 0 (new values; u_z of a 2-D lattice stays 0)
__global__ void __launch_bounds__(256) fields_plus_kernel(const double* __restrict__ oldf, const double* __restrict__ drho,
                                                          const double* __restrict__ du, const double* __restrict__ dT,
                                                          double* __restrict__ newf, long long N, int D, int keep) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const double k = keep ? 1.0 : 0.0;
  newf[n] = k * oldf[n] + drho[n];
  for (int a = 0; a < 3; ++a) newf[(1 + a) * N + n] = k * oldf[(1 + a) * N + n] + (a < D ? du[a * N + n] : 0.0);
  newf[4 * N + n] = k * oldf[4 * N + n] + dT[n];
}

// coarse node: means of rho, rho u and rho E over its factor^D fine nodes;
// T from U(T) = E - |u|^2 / 2 with the caloric law of p
__global__ void __launch_bounds__(256) filter_kernel(const double* __restrict__ fields, long long N, int nx, int ny,
                                                     int nz, int f, int fz, int D, const StepParams p,
                                                     double* __restrict__ rho, double* __restrict__ u,
                                                     double* __restrict__ T) {
  const int cx = nx / f, cy = ny / f, cz = nz / fz;
  const long long Nc = (long long)cx * cy * cz;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= Nc) return;
  const int X = (int)(c % cx), Y = (int)((c / cx) % cy), Z = (int)(c / ((long long)cx * cy));
  double sr = 0.0, sj[3] = {0.0, 0.0, 0.0}, se = 0.0;
  for (int k = 0; k < fz; ++k)
    for (int j = 0; j < f; ++j)
      for (int i = 0; i < f; ++i) {
        const long long n = (long long)(X * f + i) + nx * ((long long)(Y * f + j) + (long long)ny * (Z * fz + k));
        const double r = fields[n];
        sr += r;
        for (int a = 0; a < 3; ++a) sj[a] += r * fields[(1 + a) * N + n];
        se += fields[5 * N + n];
      }
  const double inv = 1.0 / sr;
  double u2 = 0.0;
  for (int a = 0; a < D; ++a) {
    const double ua = sj[a] * inv;
    u[a * Nc + c] = ua;
    u2 += ua * ua;
  }
  const double cnt = (double)f * f * fz;
  rho[c] = sr / cnt;
  const double e = se * inv - 0.5 * u2;
  T[c] = p.caloric ? caloric_step(p.Cv, p.cv1, p.cv2, 0.0, e) : e / p.Cv;
}

hipError_t launch_fields_add(const Ctx& c, void* pops, const double* oldf, const double* newf) {
  const long long N = c.N;
  const dim3 grid((unsigned)((N + 255) / 256)), block(256);
  if (c.lattice == 3) {
    if (c.precision == LBM_FP64)
      hipLaunchKernelGGL((fields_add_kernel<3, false, double>), grid, block, 0, c.stream, (double*)pops, oldf, newf, N,
                         c.sp);
    else
      hipLaunchKernelGGL((fields_add_kernel<3, true, float>), grid, block, 0, c.stream, (float*)pops, oldf, newf, N,
                         c.sp);
  } else {
    if (c.precision == LBM_FP64)
      hipLaunchKernelGGL((fields_add_kernel<2, false, double>), grid, block, 0, c.stream, (double*)pops, oldf, newf, N,
                         c.sp);
    else
      hipLaunchKernelGGL((fields_add_kernel<2, true, float>), grid, block, 0, c.stream, (float*)pops, oldf, newf, N,
                         c.sp);
  }
  return hipGetLastError();
}

hipError_t launch_fields_plus(const Ctx& c, const double* oldf, const double* drho, const double* du, const double* dT,
                              double* newf, bool keep) {
  const long long N = c.N;
  hipLaunchKernelGGL(fields_plus_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, c.stream, oldf, drho, du, dT,
                     newf, N, c.lattice, keep ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_filter(const Ctx& c, const double* fields, int factor, double* rho, double* u, double* T) {
  const int fz = c.lattice == 3 ? factor : 1;
  const long long Nc = (c.n[0] / factor) * (c.n[1] / factor) * (c.n[2] / fz);
  hipLaunchKernelGGL(filter_kernel, dim3((unsigned)((Nc + 255) / 256)), dim3(256), 0, c.stream, fields, c.N,
                     (int)c.n[0], (int)c.n[1], (int)c.n[2], factor, fz, c.lattice, c.sp, rho, u, T);
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
  return (int)(want < kMaxDiagBlocks ? want : kMaxDiagBlocks);
}

// Device memory of the allocation-free diagnostics (lbm_diagnostics_noalloc):
// the per-block partial sums and the final sums, kScratchDoubles doubles
// (344 KB) on every device the library runs on, held until the process
// ends.  Host code never uses this name as an address: scratch_address
// returns the device address of the current device's copy.
static __device__ __align__(256) double scratch[kScratchDoubles];

hipError_t scratch_address(double** out) {
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  *out = e == hipSuccess ? static_cast<double*>(ptr) : nullptr;
  return e;
}

hipError_t launch_diag_direct(const Ctx& c, const void* pops, double* partial, int nblocks, double* out) {
  if (c.lattice == 3) {
    if (c.precision == LBM_FP64)
      hipLaunchKernelGGL((diag_direct_kernel<3, double>), dim3(nblocks), dim3(256), 0, c.stream,
                         static_cast<const double*>(pops), partial, (long long)c.N, c.sp);
    else
      hipLaunchKernelGGL((diag_direct_kernel<3, float>), dim3(nblocks), dim3(256), 0, c.stream,
                         static_cast<const float*>(pops), partial, (long long)c.N, c.sp);
  } else {
    if (c.precision == LBM_FP64)
      hipLaunchKernelGGL((diag_direct_kernel<2, double>), dim3(nblocks), dim3(256), 0, c.stream,
                         static_cast<const double*>(pops), partial, (long long)c.N, c.sp);
    else
      hipLaunchKernelGGL((diag_direct_kernel<2, float>), dim3(nblocks), dim3(256), 0, c.stream,
                         static_cast<const float*>(pops), partial, (long long)c.N, c.sp);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((final_reduce_kernel<kNumDiag>), dim3(1), dim3(256), 0, c.stream, partial, nblocks, out);
  return hipGetLastError();
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
  // one 16-byte vector per thread; launches of at most 2^30 vectors
  const long long n16 = (long long)(bytes / 16);
  constexpr long long kMax = 1LL << 30;
  for (long long off = 0; off < n16; off += kMax) {
    const long long n = n16 - off < kMax ? n16 - off : kMax;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (const float4*)src + off,
                       (float4*)dst + off, n);
  }
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
