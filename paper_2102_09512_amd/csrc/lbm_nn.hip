// Learned coarse-grid corrector of liblbm.so: 3x3x3 periodic convolutions
// on bf16 matrix cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation),
// forward, backward-data and backward-weight kernels, the training loss and
// an FP32 Adam step.  The C ABI is in lbm_nn.h.
//
// Layouts.  Activations are bf16, channels-last: a[v][C] with v the node
// index (x fastest) and C = 16 (the network input, zero-padded) or 32 (every
// layer output, zero-padded past the layer's width).  Weights are kept in
// FP32 as W[t][i][o] (tap t = (dx+1) + 3(dy+1) + 9(dz+1)) and packed to bf16
// for the matrix cores as wp[t][i/16][o][i%16] (forward) and, for the
// gradient with respect to the layer input, as the convolution with the
// mirrored taps and exchanged channels, wb[t][o/16][i][o%16].
//
// Matrix-core tiles (v_mfma_f32_32x32x16_bf16: lane l supplies
// A[m = l%32][k = 8(l/32) .. +7] and B[k = 8(l/32) .. +7][n = l%32];
// accumulator i of lane l holds C[m = 8(i/4) + 4(l/32) + i%4][n = l%32]).
// Convolution: A = weights (m = output channel, k = input channel), B =
// activations (n = node of a 32-node row), so a lane ends with four
// consecutive output channels of one node per accumulator group.  Weight
// gradient: A = input activations (m = input channel, k = node), B = output
// gradient (n = output channel), summed over nodes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbm_internal.h"
#include "lbm_nn.h"

namespace lbmnn {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef float f4v __attribute__((ext_vector_type(4)));

struct Grid {
  int nx, ny, nz;
};

__device__ inline int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// planar FP32 x[c][v] (c < cin) -> bf16 a[v][16], (x - mean) / std, zero padded
__global__ void __launch_bounds__(256) pack_input_kernel(const float* __restrict__ x, int cin, const float* __restrict__ mean,
                                                         const float* __restrict__ inv_std, __bf16* __restrict__ a, int V) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  bf8 lo, hi;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    lo[c] = (__bf16)(c < cin ? (x[(size_t)c * V + v] - mean[c]) * inv_std[c] : 0.f);
    hi[c] = (__bf16)(c + 8 < cin ? (x[(size_t)(c + 8) * V + v] - mean[c + 8]) * inv_std[c + 8] : 0.f);
  }
  *(bf8*)(a + (size_t)v * 16) = lo;
  *(bf8*)(a + (size_t)v * 16 + 8) = hi;
}

// Output tile of the convolution kernel: 32 nodes along x (the matrix-core
// N dimension) times kTY rows along y times kTZ planes along z; row q of the
// tile is (y0 + q % kTY, z0 + q / kTY) and wave w computes rows w kR ..
// w kR + kR - 1.  The input tile with its one-node periodic halo is staged in
// LDS once per block and read 27 times.
constexpr int kTX = 32, kTY = 4, kTZ = 4;
constexpr int kW = 4;                   // wavefronts per work-group (3% faster than 8: each weight operand serves 4 rows)
constexpr int kR = kTY * kTZ / kW;      // output rows (32 nodes each) per wavefront
constexpr int kHX = kTX + 2, kHY = kTY + 2, kHZ = kTZ + 2;

// Consecutive hardware work-group ids go round the eight XCDs (each with its
// own L2); the logical tile order is rebuilt so that every XCD runs one
// contiguous range of tiles, whose halos then overlap inside that XCD's L2.
__device__ inline int xcd_tile(int b, int nblocks) {
  const int q8 = nblocks >> 3, r8 = nblocks & 7, xcd = b & 7;
  return xcd * q8 + min(xcd, r8) + (b >> 3);
}

// 16-byte chunk c of the node at halo column hx is stored at chunk
// c ^ f(hx).  A 16-byte LDS read is served sixteen lanes at a time over 64
// banks of 4 bytes (256 bytes); sixteen consecutive lanes (consecutive hx,
// same c, any alignment) then hit sixteen disjoint groups of four banks.
// (The swizzle that is conflict-free for eight lanes over 32 banks,
// c ^ ((hx >> 1) & 3), measured 46% of the LDS cycles as bank conflicts.)
template <int CIN>
__device__ inline int swizzle(int c, int hx) {
  return CIN == 32 ? (c ^ ((hx >> 2) & 3)) : (c ^ ((hx >> 3) & 1));
}

// out[v][o] = bias[o] + sum_t sum_i in[v + s_t][i] w[t][i][o]  (cross-correlation)
// as the product W^T (32 outputs x K) times the input columns (K x 32 nodes),
// K = 27 taps x CIN: A[m = o][k = i] from wp, B[k = i][n = node] from LDS;
// accumulator i of lane l holds output channel 8(i/4) + 4(l/32) + i%4 of node
// x0 + l%32.  CIN: channels of in (16 or 32).  OUT_PLANAR: FP32 planes
// out[o][v] for o < cout, else bf16 out[v][32].  relu: max(., 0).  mask (bf16
// [v][32], may be null): zero where mask <= 0 (the derivative of the ReLU that
// produced it).  bias may be null; it holds cout values.
// Requires nx % 32 == 0, ny % 4 == 0, nz % 4 == 0; grid = tiles.
// Stages the input tile of output tile (x0, y0, z0) with its one-node
// periodic halo in LDS, swizzled (every thread issues all its loads before
// its first LDS write, so the tile costs one memory latency instead of one
// per chunk), and waits for the work-group.
template <int CIN>
__device__ inline void stage_tile(const __bf16* __restrict__ in, __bf16* tile, const Grid& g, int x0, int y0, int z0) {
  constexpr int CH = CIN / 8;                           // 16-byte chunks per node
  constexpr int NCH = kHZ * kHY * kHX * CH;            // 16-byte chunks of the halo tile
  constexpr int NIT = (NCH + 64 * kW - 1) / (64 * kW);  // chunks per thread
  bf8 stage[NIT];
#pragma unroll
  for (int k = 0; k < NIT; ++k) {
    const int e = threadIdx.x + k * 64 * kW;
    if (e < NCH) {
      const int c = e % CH, node = e / CH;
      const int hx = node % kHX, hy = (node / kHX) % kHY, hz = node / (kHX * kHY);
      const int gx = wrap(x0 + hx - 1, g.nx), gy = wrap(y0 + hy - 1, g.ny), gz = wrap(z0 + hz - 1, g.nz);
      stage[k] = *(const bf8*)(in + (size_t)(gx + g.nx * (gy + g.ny * gz)) * CIN + c * 8);
    }
  }
#pragma unroll
  for (int k = 0; k < NIT; ++k) {
    const int e = threadIdx.x + k * 64 * kW;
    if (e < NCH) {
      const int c = e % CH, node = e / CH;
      *(bf8*)(tile + node * CIN + swizzle<CIN>(c, node % kHX) * 8) = stage[k];
    }
  }
  __syncthreads();
}

// Bias, ReLU, ReLU-derivative mask and store of a wavefront's kR output rows
// (32 x 32 accumulator layout: accumulator i of lane l holds output channel
// 8(i/4) + 4(l/32) + i%4 of node x0 + l%32).
template <bool OUT_PLANAR>
__device__ inline void conv_epilogue(const f16v* acc, const float* bo, int relu, const __bf16* __restrict__ mask,
                                     void* __restrict__ out, int cout, const Grid& g, int V, int x0, int y0, int z0,
                                     int w, int r, int half) {
#pragma unroll
  for (int j = 0; j < kR; ++j) {
    const int q = w * kR + j;
    const int v = (x0 + r) + g.nx * ((y0 + q % kTY) + g.ny * (z0 + q / kTY));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c0 = 8 * q + 4 * half;
      float y[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        y[k] = acc[j][4 * q + k] + bo[4 * q + k];
        if (relu) y[k] = y[k] > 0.f ? y[k] : 0.f;
      }
      if (mask) {
        typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
        const bf4 mk = *(const bf4*)(mask + (size_t)v * 32 + c0);
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (!((float)mk[k] > 0.f)) y[k] = 0.f;
      }
      if (OUT_PLANAR) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (c0 + k < cout) static_cast<float*>(out)[(size_t)(c0 + k) * V + v] = y[k];
      } else {
        typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
        bf4 o;
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = (__bf16)y[k];
        *(bf4*)(static_cast<__bf16*>(out) + (size_t)v * 32 + c0) = o;
      }
    }
  }
}

template <int CIN, bool OUT_PLANAR>
__global__ void __launch_bounds__(64 * kW) conv_kernel(const __bf16* __restrict__ in, const __bf16* __restrict__ wp,
                                                   const float* __restrict__ bias, int relu,
                                                   const __bf16* __restrict__ mask, void* __restrict__ out, int cout,
                                                   const Grid g, int V) {
  __shared__ __attribute__((aligned(16))) __bf16 tile[kHZ * kHY * kHX * CIN];
  const int tx = g.nx / kTX, ty = g.ny / kTY;
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (b % tx) * kTX, y0 = ((b / tx) % ty) * kTY, z0 = (b / (tx * ty)) * kTZ;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 31, half = lane >> 5;
  // Wave w owns the kTY output rows of plane z = w of the tile.  For one
  // (dz, dx) pair and 16-channel block, each of the kTY + 2 input rows of
  // the halo column is read from LDS once and feeds the (up to three)
  // output rows it reaches through the taps dy = -1, 0, 1, each with its own
  // weights: half the LDS reads of one read per tap and row.  The weights of
  // group (dz, dx) come from L2 while the group before it computes (two
  // register sets, one group of matrix-core work ahead); the first group's
  // and the biases are requested before the tile is staged.
  static_assert(kR == kTY && kW == kTZ, "a wavefront owns one plane of the tile");
  constexpr int NC = CIN / 16;
  bf8 a[2][NC][3];  // [set][16-channel block][dy + 1]
  auto load_group = [&](int gi, bf8(&dst)[NC][3]) {
    const int dz = gi / 3 - 1, dx = gi % 3 - 1;
#pragma unroll
    for (int cc = 0; cc < NC; ++cc)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int t = (dx + 1) + 3 * k + 9 * (dz + 1);
        dst[cc][k] = *(const bf8*)(wp + ((size_t)(t * NC + cc) * 32 + r) * 16 + 8 * half);
      }
  };
  load_group(0, a[0]);
  float bo[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int c = 8 * (i >> 2) + 4 * half + (i & 3);
    bo[i] = bias && c < cout ? bias[c] : 0.f;
  }
  stage_tile<CIN>(in, tile, g, x0, y0, z0);
  f16v acc[kR] = {};
#pragma unroll
  for (int gi = 0; gi < 9; ++gi) {
    if (gi + 1 < 9) load_group(gi + 1, a[(gi + 1) & 1]);
    __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of this group's work
    const int dz = gi / 3 - 1, dx = gi % 3 - 1;
    const int hz = w + dz + 1, hx = r + dx + 1;
    const __bf16* col = tile + hx * CIN + hz * kHY * kHX * CIN;
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
      const int off = swizzle<CIN>(2 * cc + half, hx) * 8;
#pragma unroll
      for (int hy = 0; hy < kTY + 2; ++hy) {
        const bf8 bv = *(const bf8*)(col + hy * kHX * CIN + off);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int j = hy - k;  // output row reached through dy = k - 1
          if (j >= 0 && j < kTY)
            acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[gi & 1][cc][k], bv, acc[j], 0, 0, 0);
        }
      }
    }
  }
  conv_epilogue<OUT_PLANAR>(acc, bo, relu, mask, out, cout, g, V, x0, y0, z0, w, r, half);
}

// Input layer of at most 8 channels (the corrector's 5: rho, u, T): the
// input activations hold 16 channels per node of which the first 8 are
// staged (16 bytes per node), and the matrix-core K dimension of 16 takes two
// taps at a time, 8 channels each: lane half h supplies tap 2p + h of pair p.
// 14 products per output row instead of 27.  wq[p][o][k]: k < 8 channel k
// of tap 2p, k >= 8 channel k - 8 of tap 2p + 1 (tap 27 does not exist: its
// weights are zero and its B operand repeats tap 26).  Output as
// conv_kernel (bf16 [v][32]).  PLANAR_IN: the input is read straight from
// the FP32 planes x[c][v] (c < cin) and normalised as pack_input_kernel does
// (the same expression, so the staged bf16 values are the same), for calls
// that need no packed copy of it (inference).
template <bool PLANAR_IN>
__global__ void __launch_bounds__(64 * kW) conv_pair_kernel(const __bf16* __restrict__ in,
                                                            const float* __restrict__ x, int cin,
                                                            const float* __restrict__ mean,
                                                            const float* __restrict__ inv_std,
                                                            const __bf16* __restrict__ wq,
                                                            const float* __restrict__ bias, int relu,
                                                            __bf16* __restrict__ out, int cout, const Grid g, int V) {
  constexpr int NN = kHZ * kHY * kHX;  // halo nodes; one 16-byte chunk each
  __shared__ __attribute__((aligned(16))) __bf16 tile[NN * 8];
  const int tx = g.nx / kTX, ty = g.ny / kTY;
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (b % tx) * kTX, y0 = ((b / tx) % ty) * kTY, z0 = (b / (tx * ty)) * kTZ;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 31, half = lane >> 5;
  // every weight operand and the biases are requested before the staging
  bf8 a[14];
#pragma unroll
  for (int p = 0; p < 14; ++p) a[p] = *(const bf8*)(wq + ((size_t)p * 32 + r) * 16 + 8 * half);
  float bo[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int c = 8 * (i >> 2) + 4 * half + (i & 3);
    bo[i] = bias && c < cout ? bias[c] : 0.f;
  }
  if constexpr (PLANAR_IN) {
    // Rows (hy, hz) of the halo block: the 32 interior nodes of a row are 8
    // aligned groups of 4 consecutive x (one 16-byte load per channel; x0
    // and nx are multiples of 32), its two end nodes (x0 - 1 and x0 + 32,
    // wrapped) are loaded one by one.
    constexpr int PER_ROW = kTX / 4 + 2, ITEMS = kHZ * kHY * PER_ROW;
    constexpr int NIT = (ITEMS + 64 * kW - 1) / (64 * kW);
    float4 xs[NIT][8];
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int item = threadIdx.x + k * 64 * kW;
      if (item < ITEMS) {
        const int row = item / PER_ROW, e = item % PER_ROW, hy = row % kHY, hz = row / kHY;
        const int gy = wrap(y0 + hy - 1, g.ny), gz = wrap(z0 + hz - 1, g.nz);
        const int gx = e < kTX / 4 ? x0 + 4 * e : wrap(e == kTX / 4 ? x0 - 1 : x0 + kTX, g.nx);
        const size_t v = (size_t)gx + (size_t)g.nx * (gy + (size_t)g.ny * gz);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          xs[k][c] = float4{0.f, 0.f, 0.f, 0.f};
          if (c < cin) {
            if (e < kTX / 4) xs[k][c] = *(const float4*)(x + (size_t)c * V + v);
            else xs[k][c].x = x[(size_t)c * V + v];
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int item = threadIdx.x + k * 64 * kW;
      if (item < ITEMS) {
        const int row = item / PER_ROW, e = item % PER_ROW;
        const int base = row * kHX;  // node index of hx = 0 in this row
        // normalised as pack_input_kernel does (the same expression, so the staged bf16 values are the same)
        auto node_chunk = [&](int n) {
          bf8 val;
#pragma unroll
          for (int c = 0; c < 8; ++c) val[c] = (__bf16)(c < cin ? (xs[k][c][n] - mean[c]) * inv_std[c] : 0.f);
          return val;
        };
        if (e < kTX / 4) {
#pragma unroll
          for (int n = 0; n < 4; ++n) *(bf8*)(tile + (base + 4 * e + n + 1) * 8) = node_chunk(n);
        } else {
          *(bf8*)(tile + (base + (e == kTX / 4 ? 0 : kHX - 1)) * 8) = node_chunk(0);
        }
      }
    }
    __syncthreads();
  } else {
    constexpr int NIT = (NN + 64 * kW - 1) / (64 * kW);
    bf8 stage[NIT];
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int node = threadIdx.x + k * 64 * kW;
      if (node < NN) {
        const int hx = node % kHX, hy = (node / kHX) % kHY, hz = node / (kHX * kHY);
        const int gx = wrap(x0 + hx - 1, g.nx), gy = wrap(y0 + hy - 1, g.ny), gz = wrap(z0 + hz - 1, g.nz);
        stage[k] = *(const bf8*)(in + ((size_t)gx + (size_t)g.nx * (gy + (size_t)g.ny * gz)) * 16);
      }
    }
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int node = threadIdx.x + k * 64 * kW;
      if (node < NN) *(bf8*)(tile + node * 8) = stage[k];
    }
    __syncthreads();
  }
  f16v acc[kR] = {};
#pragma unroll
  for (int p = 0; p < 14; ++p) {
    const int t = min(2 * p + half, 26);
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    const __bf16* col = tile + (r + dx + 1) * 8;
#pragma unroll
    for (int j = 0; j < kR; ++j) {
      const int q = w * kR + j, hy = q % kTY + dy + 1, hz = q / kTY + dz + 1;
      const bf8 bv = *(const bf8*)(col + (hz * kHY + hy) * kHX * 8);
      acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[p], bv, acc[j], 0, 0, 0);
    }
  }
  conv_epilogue<false>(acc, bo, relu, nullptr, out, cout, g, V, x0, y0, z0, w, r, half);
}

// Output layer with at most 16 channels (the corrector's 3): the same
// convolution on v_mfma_f32_16x16x32_bf16 (A 16 x 32, B 32 x 16; lane l
// supplies A[l%16][8(l/16) .. +7] and B[8(l/16) .. +7][l%16] and holds
// D[4(l/16) .. +3][l%16]), with A = weights (m = output channel, padded to
// 16 instead of 32, k = the 32 input channels of one tap) and B = the
// activations of 16 nodes: half the matrix-core work of conv_kernel for such
// a layer.  FP32 planes out[o][v] for o < cout.  wn[t][o][i] (o < 16,
// i < 32).  Same tile and staging as conv_kernel; input width 32.
__global__ void __launch_bounds__(64 * kW) conv_narrow_kernel(const __bf16* __restrict__ in,
                                                              const __bf16* __restrict__ wn,
                                                              const float* __restrict__ bias,
                                                              float* __restrict__ out, int cout, const Grid g, int V) {
  __shared__ __attribute__((aligned(16))) __bf16 tile[kHZ * kHY * kHX * 32];
  const int tx = g.nx / kTX, ty = g.ny / kTY;
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (b % tx) * kTX, y0 = ((b / tx) % ty) * kTY, z0 = (b / (tx * ty)) * kTZ;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n16 = lane & 15, grp = lane >> 4;
  // weights of group (dz, dx), taps dy = -1, 0, 1: A[o = l%16][i = 8(l/16) + j];
  // one group ahead, as in conv_kernel
  bf8 a[2][3];
  auto load_group = [&](int gi, bf8(&dst)[3]) {
    const int dz = gi / 3 - 1, dx = gi % 3 - 1;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int t = (dx + 1) + 3 * k + 9 * (dz + 1);
      dst[k] = *(const bf8*)(wn + ((size_t)t * 16 + n16) * 32 + 8 * grp);
    }
  };
  load_group(0, a[0]);
  float bo[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) bo[v] = bias && 4 * grp + v < cout ? bias[4 * grp + v] : 0.f;
  stage_tile<32>(in, tile, g, x0, y0, z0);
  f4v acc[kTY][2] = {};
#pragma unroll
  for (int gi = 0; gi < 9; ++gi) {
    if (gi + 1 < 9) load_group(gi + 1, a[(gi + 1) & 1]);
    __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of this group's work
    const int dz = gi / 3 - 1, dx = gi % 3 - 1;
    const int hz = w + dz + 1;
#pragma unroll
    for (int hy = 0; hy < kTY + 2; ++hy) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int hx = 16 * h + n16 + dx + 1;
        const bf8 bv = *(const bf8*)(tile + ((hz * kHY + hy) * kHX + hx) * 32 + swizzle<32>(grp, hx) * 8);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int j = hy - k;
          if (j >= 0 && j < kTY)
            acc[j][h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[gi & 1][k], bv, acc[j][h], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kTY; ++j)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int v = (x0 + 16 * h + n16) + g.nx * ((y0 + j) + g.ny * (z0 + w));
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = 4 * grp + q;
        if (c < cout) out[(size_t)c * V + v] = acc[j][h][q] + bo[q];
      }
    }
}

// Weight and bias gradients of one layer, per work-group partial sums over
// the layer's real channels (i < cin, o < cout):
//   slot t < 27: part[t][b][i][o] = sum over the group's nodes v of in[v + s_t][i] dout[v][o]
//   slot 27:     part[27][b][i][o] = sum over the group's nodes v of dout[v][o] (every row i)
// (the bias gradient as the product with a row of ones).  Work-group b takes
// tiles b tpb .. b tpb + tpb - 1 of 32 x 4 x 2 nodes (x fastest, then y, z).
// Per tile the input with its one-node halo and the output gradient are
// staged in LDS channel-major, so that the node index runs along the
// matrix-core K dimension: lane (r, h) reads 8 consecutive nodes of channel r
// as one 16-byte word.  The x offset of a tap is 0, 1 or 2 elements inside
// two aligned words and is taken out with funnel shifts.  Wave w owns seven
// slots (the three dx taps of two (dy, dz) pairs and one more; see the loop)
// and keeps their sums in registers across the tiles.
constexpr int kGX = 32, kGY = 4, kGZ = 2;
constexpr int kGHY = kGY + 2, kGHZ = kGZ + 2, kGHX = kGX + 2;
constexpr int kGRow = 40;                           // halo row: 34 nodes, padded to a 16-byte multiple
constexpr int kGPlaneIn = kGHZ * kGHY * kGRow + 8;  // per channel; the 16 extra bytes spread the
constexpr int kGPlaneD = kGZ * kGY * kGX + 8;       // channel planes over the LDS banks
constexpr int kGMaxBlocks = 512;
constexpr int kGSegments = 16;  // first-stage runs of the gradient sum

typedef unsigned int u4 __attribute__((ext_vector_type(4)));

template <int CIN>
__global__ void __launch_bounds__(256) wgrad_kernel(const __bf16* __restrict__ in, const __bf16* __restrict__ dout,
                                                    float* __restrict__ part, const Grid g, int ntiles, int tpb,
                                                    int cin, int cout) {
  __shared__ __attribute__((aligned(16))) __bf16 inT[CIN * kGPlaneIn];
  __shared__ __attribute__((aligned(16))) __bf16 dT[32 * kGPlaneD];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 31, half = lane >> 5;
  const int tx = g.nx / kGX, ty = g.ny / kGY;
  bf8 ones;
#pragma unroll
  for (int j = 0; j < 8; ++j) ones[j] = (__bf16)1.f;
  f16v acc[7] = {};
  const int bl = xcd_tile(blockIdx.x, gridDim.x);  // logical block: tiles and partial slot
  const int first = bl * tpb, last = min(first + tpb, ntiles);
  for (int tile = first; tile < last; ++tile) {
    const int x0 = (tile % tx) * kGX, y0 = ((tile / tx) % ty) * kGY, z0 = (tile / (tx * ty)) * kGZ;
    __syncthreads();  // every wave is done with the previous tile
    constexpr int NH = kGHX * kGHY * kGHZ;
    for (int e = threadIdx.x; e < NH * (CIN / 8); e += 256) {
      const int node = e % NH, c8 = e / NH;
      const int hx = node % kGHX, hy = (node / kGHX) % kGHY, hz = node / (kGHX * kGHY);
      const int gx = wrap(x0 + hx - 1, g.nx), gy = wrap(y0 + hy - 1, g.ny), gz = wrap(z0 + hz - 1, g.nz);
      const bf8 val = *(const bf8*)(in + (size_t)(gx + g.nx * (gy + g.ny * gz)) * CIN + 8 * c8);
      __bf16* dst = inT + 8 * c8 * kGPlaneIn + (hz * kGHY + hy) * kGRow + hx;
#pragma unroll
      for (int j = 0; j < 8; ++j) dst[j * kGPlaneIn] = val[j];
    }
    constexpr int ND = kGX * kGY * kGZ;
    for (int e = threadIdx.x; e < ND * 4; e += 256) {
      const int node = e % ND, c8 = e / ND;
      const int xx = node % kGX, yy = (node / kGX) % kGY, zz = node / (kGX * kGY);
      const bf8 val = *(const bf8*)(dout + (size_t)((x0 + xx) + g.nx * ((y0 + yy) + g.ny * (z0 + zz))) * 32 + 8 * c8);
      __bf16* dst = dT + 8 * c8 * kGPlaneD + node;
#pragma unroll
      for (int j = 0; j < 8; ++j) dst[j * kGPlaneD] = val[j];
    }
    __syncthreads();
    // The three slots of one (dy, dz) pair (dx = -1, 0, 1) read the same two
    // words of a channel row and differ by a shift of 0, 1 or 2 elements, so a
    // wave owns whole pairs: wave w takes the pairs 2w and 2w + 1 (slots 6w ..
    // 6w + 5) and a seventh slot, dx = w - 1 of pair 8 (slot 24 + w) for w < 3
    // and the bias (slot 27) for w = 3.  Two LDS reads serve three products.
#pragma unroll 1
    for (int row = 0; row < kGY * kGZ; ++row) {
      const int yy = row % kGY, zz = row / kGY;
#pragma unroll
      for (int kb = 0; kb < kGX; kb += 16) {
        // the output gradient of these 16 nodes serves all seven slots of the wave
        const bf8 b = *(const bf8*)(dT + r * kGPlaneD + (zz * kGY + yy) * kGX + kb + 8 * half);
        auto words = [&](int pair, u4& lo, u4& hi) {
          const int dy = pair % 3 - 1, dz = pair / 3 - 1;
          const __bf16* src = inT + r * kGPlaneIn + ((zz + dz + 1) * kGHY + yy + dy + 1) * kGRow + kb + 8 * half;
          lo = *(const u4*)src;
          hi = *(const u4*)(src + 8);
        };
        auto shifted = [&](const u4& lo, const u4& hi, int o) {  // the 8 elements from element o of lo
          u4 v;
          if (o == 0) {
            v = lo;
          } else if (o == 2) {
            v = u4{lo.y, lo.z, lo.w, hi.x};
          } else {
            v = u4{__builtin_amdgcn_alignbit(lo.y, lo.x, 16), __builtin_amdgcn_alignbit(lo.z, lo.y, 16),
                   __builtin_amdgcn_alignbit(lo.w, lo.z, 16), __builtin_amdgcn_alignbit(hi.x, lo.w, 16)};
          }
          return __builtin_bit_cast(bf8, v);
        };
#pragma unroll
        for (int gp = 0; gp < 2; ++gp) {
          u4 lo{}, hi{};
          if (r < CIN) words(2 * w + gp, lo, hi);
#pragma unroll
          for (int o = 0; o < 3; ++o)
            acc[3 * gp + o] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(shifted(lo, hi, o), b, acc[3 * gp + o], 0, 0, 0);
        }
        bf8 a = ones;
        if (w < 3) {
          u4 lo{}, hi{};
          if (r < CIN) words(8, lo, hi);
          a = shifted(lo, hi, w);
        }
        acc[6] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[6], 0, 0, 0);
      }
    }
  }
  // accumulator i of lane l holds input channel m = 8(i/4) + 4(l/32) + i%4
  // and output channel r = l%32
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const int t = k < 6 ? 6 * w + k : (w < 3 ? 24 + w : 27);
    float* dst = part + ((size_t)t * gridDim.x + bl) * cin * cout;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int m = 8 * (i >> 2) + 4 * half + (i & 3);
      if (m < cin && r < cout) dst[m * cout + r] = acc[k][i];
    }
  }
}

// src[0] + src[stride] + ... + src[(n - 1) stride], added in that order, with
// eight loads in flight at a time.
__device__ inline float ordered_sum(const float* __restrict__ src, size_t stride, int n) {
  float acc = 0.f;
  int b = 0;
  for (; b + 8 <= n; b += 8) {
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = src[(size_t)(b + j) * stride];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += v[j];
  }
  for (; b < n; ++b) acc += src[(size_t)b * stride];
  return acc;
}

// First stage of the gradient sum: part2[t][s][io] = sum of part[t][b][io]
// over the s-th of nseg equal runs of b (blockIdx.y = s), io < cio = cin
// cout; fixed order.
__global__ void __launch_bounds__(256) wgrad_partial_sum_kernel(const float* __restrict__ part, int nblk, int nseg,
                                                                int cio, float* __restrict__ part2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 28 * cio) return;
  const int t = e / cio, io = e % cio, sgm = blockIdx.y;
  const int b0 = (int)((long long)nblk * sgm / nseg), b1 = (int)((long long)nblk * (sgm + 1) / nseg);
  part2[((size_t)t * nseg + sgm) * cio + io] = ordered_sum(part + ((size_t)t * nblk + b0) * cio + io, cio, b1 - b0);
}

// grad[t][i][o] += sum_b part[t][b][i][o] (t < 27) and grad_b[o] += sum_b
// part[27][b][0][o], part laid out [28][nblk][cin][cout]; fixed summation order
__global__ void __launch_bounds__(256) wgrad_reduce_kernel(const float* __restrict__ part, int nblk, int cin, int cout,
                                                           float* __restrict__ grad, float* __restrict__ grad_b) {
  const int cio = cin * cout;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 28 * cio) return;
  const int t = e / cio, io = e % cio, i = io / cout, o = io % cout;
  if (t == 27 && i != 0) return;
  const float s = ordered_sum(part + (size_t)t * nblk * cio + io, cio, nblk);
  if (t < 27) grad[((size_t)t * cin + i) * cout + o] += s;
  else grad_b[o] += s;
}

// r_c = y_c + (x_f - target_f) / out_std_c with f = off + c; loss partial sums
// of r^2; dout[v][c] = 2 r / (C V)
__global__ void __launch_bounds__(256) loss_kernel(const float* __restrict__ y, const float* __restrict__ x,
                                                   const float* __restrict__ tgt, const float* __restrict__ inv_std,
                                                   int C, int off, int V, __bf16* __restrict__ dout,
                                                   double* __restrict__ partial) {
  __shared__ double red[256];
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (v < V) {
    const float scale = 2.f / ((float)C * (float)V);
    bf8 o[4];  // the node's 32 gradient channels, stored as four 16-byte words
#pragma unroll
    for (int c = 0; c < 32; ++c) {
      float g = 0.f;
      if (c < C) {
        const size_t f = (size_t)(off + c) * V + v;
        const float rr = y[(size_t)c * V + v] + (x[f] - tgt[f]) * inv_std[c];
        s += (double)rr * rr;
        g = scale * rr;
      }
      o[c / 8][c % 8] = (__bf16)g;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) *(bf8*)(dout + (size_t)v * 32 + 8 * q) = o[q];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// acc[0] += scale * (sum of partial[0 .. n-1]) in a fixed order (one
// work-group): the loss of one sample added to a device-side running sum.
__global__ void __launch_bounds__(256) loss_accumulate_kernel(const double* __restrict__ partial, int n, double scale,
                                                              double* __restrict__ acc) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) acc[0] += scale * red[0];
}

__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, long long n, float lr,
                                                   float b1, float b2, float eps, float gscale, float c1, float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i] * gscale;
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// bf16 copies of one layer's FP32 weights W[t][i][o] (cin x cout):
// wp[t][i/16][o][i%16] (CINP padded inputs, 32 outputs) and
// wb[t][o/16][i][o%16] = W[26 - t][i][o] (32 padded outputs as inputs, 32 rows)
// and, for an output layer of at most 16 channels, wn[t][o][i] = W[t][i][o]
// (16 padded outputs, 32 padded inputs); for an input layer of at most 8
// channels, wq[p][o][k] (taps 2p and 2p + 1, 8 channels each)
__global__ void __launch_bounds__(256) pack_weights_kernel(const float* __restrict__ W, int cin, int cout, int cinp,
                                                           __bf16* __restrict__ wp, __bf16* __restrict__ wb,
                                                           __bf16* __restrict__ wn, __bf16* __restrict__ wq) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < 27 * cinp * 32) {  // wp element (t, cc, o, k)
    const int k = e % 16, o = (e / 16) % 32, cc = (e / 512) % (cinp / 16), t = e / (512 * (cinp / 16));
    const int i = cc * 16 + k;
    wp[e] = (__bf16)(i < cin && o < cout ? W[((size_t)t * cin + i) * cout + o] : 0.f);
  }
  if (wq && e < 14 * 32 * 16) {  // wq element (p, o, k): tap 2p + k / 8, channel k % 8
    const int k = e % 16, o = (e / 16) % 32, p = e / 512;
    const int t = 2 * p + k / 8, i = k % 8;
    wq[e] = (__bf16)(t < 27 && i < cin && o < cout ? W[((size_t)t * cin + i) * cout + o] : 0.f);
  }
  if (wn && e < 27 * 16 * 32) {  // wn element (t, o, i)
    const int i = e % 32, o = (e / 32) % 16, t = e / 512;
    wn[e] = (__bf16)(i < cin && o < cout ? W[((size_t)t * cin + i) * cout + o] : 0.f);
  }
  if (wb && e < 27 * 32 * 32) {  // wb element (t, oc, i, k): input channel of the mirrored conv = o
    const int k = e % 16, i = (e / 16) % 32, oc = (e / 512) % 2, t = e / 1024;
    const int o = oc * 16 + k;
    wb[e] = (__bf16)(i < cin && o < cout ? W[((size_t)(26 - t) * cin + i) * cout + o] : 0.f);
  }
}

// FP64 fields of a lattice Boltzmann handle (rho, u planes, T) -> FP32 planes
__global__ void __launch_bounds__(256) fields_to_input_kernel(const double* __restrict__ rho, const double* __restrict__ u,
                                                              const double* __restrict__ T, int D, int V,
                                                              float* __restrict__ x) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  x[v] = (float)rho[v];
  for (int a = 0; a < D; ++a) x[(size_t)(1 + a) * V + v] = (float)u[(size_t)a * V + v];
  x[(size_t)(1 + D) * V + v] = (float)T[v];
}

// normalised correction planes -> FP64 increments drho[V], du[D V], dT[V]:
// output c corrects field off + c (0 rho, 1..D u, D + 1 T); fields without an
// output get a zero increment; with limit > 0 the normalised output is
// clipped to [-limit, limit] first
__global__ void __launch_bounds__(256) output_to_increments_kernel(const float* __restrict__ y,
                                                                   const float* __restrict__ sd, int C, int off, int D,
                                                                   float limit, int V, double* __restrict__ drho,
                                                                   double* __restrict__ du, double* __restrict__ dT) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  for (int fld = 0; fld < D + 2; ++fld) {
    const int c = fld - off;
    float yc = (c >= 0 && c < C) ? y[(size_t)c * V + v] : 0.f;
    if (limit > 0.f) yc = fminf(fmaxf(yc, -limit), limit);
    const double inc = (c >= 0 && c < C) ? (double)yc * sd[c] : 0.0;
    if (fld == 0) drho[v] = inc;
    else if (fld <= D) du[(size_t)(fld - 1) * V + v] = inc;
    else dT[v] = inc;
  }
}

}  // namespace lbmnn

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

namespace {

int nn_fail(int code, const std::string& msg) { return lbm::set_error(code, msg); }

int nn_hip(hipError_t e, const char* what) {
  return nn_fail(LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define NN_HIP(expr, what)                            \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return nn_hip(e_, what);    \
  } while (0)

struct Layer {
  int cin, cout, cinp;          // channels, padded input channels (16 or 32)
  long long w_off, b_off;       // offsets in the parameter vector
  __bf16 *wp = nullptr, *wb = nullptr;
  __bf16* wn = nullptr;         // output layer of <= 16 channels from 32 inputs: weights for conv_narrow_kernel
  __bf16* wq = nullptr;         // input layer of <= 8 channels (not the last): weights for conv_pair_kernel
};

}  // namespace

struct lbm_nn_ctx {
  int L = 0;
  std::vector<int> ch;
  lbmnn::Grid g{};
  int V = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  std::vector<Layer> layers;
  long long nparam = 0;
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
  float *mean = nullptr, *inv_std = nullptr;          // input scaling (device, 16 each)
  float *out_std = nullptr, *inv_out_std = nullptr;   // output scaling (device, 32 each)
  std::vector<__bf16*> act;     // act[l]: input of layer l (bf16 [V][16 or 32]); act[L] unused
  __bf16 *dA = nullptr, *dB = nullptr;  // gradient ping-pong, bf16 [V][32]
  float* y = nullptr;                   // network output planes [c_L][V]
  float* part = nullptr;                // weight-gradient partials, per work-group
  float* part2 = nullptr;               // their first-stage sums
  int out_off = 0;                      // output c corrects / is compared with field out_off + c
  double limit = 0.0;                   // lbm_nn_correct clips outputs to [-limit, limit] (0: no clip)
  double* lpart = nullptr;              // loss partials
  double* loss_acc = nullptr;           // running sum of asynchronous losses (device, 1 value)
  long long loss_count = 0;             // losses added to it since the last lbm_nn_take_loss
  float* fld = nullptr;                 // corrector staging: fields and correction (FP32)
  double* dfld = nullptr;               // FP64 fields / increments for lbm
};

namespace {

int nn_select(lbm_nn n) {
  int cur = -1;
  NN_HIP(hipGetDevice(&cur), "hipGetDevice");
  if (cur != n->device) NN_HIP(hipSetDevice(n->device), "hipSetDevice");
  return LBM_OK;
}

int nn_pack_weights(lbm_nn n) {
  for (int l = 0; l < n->L; ++l) {
    Layer& ly = n->layers[l];
    const int total = 27 * 32 * 32 > 27 * ly.cinp * 32 ? 27 * 32 * 32 : 27 * ly.cinp * 32;
    hipLaunchKernelGGL(lbmnn::pack_weights_kernel, dim3((total + 255) / 256), dim3(256), 0, n->stream,
                       n->params + ly.w_off, ly.cin, ly.cout, ly.cinp, ly.wp, l > 0 ? ly.wb : nullptr, ly.wn, ly.wq);
    NN_HIP(hipGetLastError(), "pack weights");
  }
  return LBM_OK;
}

template <int CIN, bool PLANAR>
hipError_t conv(lbm_nn n, const __bf16* in, const __bf16* w, const float* bias, int relu, const __bf16* mask,
                void* out, int cout) {
  const int blocks = (n->g.nx / lbmnn::kTX) * (n->g.ny / lbmnn::kTY) * (n->g.nz / lbmnn::kTZ);
  hipLaunchKernelGGL((lbmnn::conv_kernel<CIN, PLANAR>), dim3(blocks), dim3(64 * lbmnn::kW), 0, n->stream, in, w, bias,
                     relu,
                     mask, out, cout, n->g, n->V);
  return hipGetLastError();
}

// forward pass of normalised x into yout (n->y if null); activations kept
// for the backward pass.  keep_input: also keep the packed input (the weight
// gradient of the first layer reads it); without it a first layer of at most
// 8 channels reads x directly.
int nn_forward(lbm_nn n, const float* x, float* yout = nullptr, bool keep_input = true) {
  if (!yout) yout = n->y;
  const bool direct = !keep_input && n->layers[0].wq && n->L > 1;
  if (!direct) {
    hipLaunchKernelGGL(lbmnn::pack_input_kernel, dim3((n->V + 255) / 256), dim3(256), 0, n->stream, x, n->ch[0],
                       n->mean, n->inv_std, n->act[0], n->V);
    NN_HIP(hipGetLastError(), "pack input");
  }
  for (int l = 0; l < n->L; ++l) {
    const Layer& ly = n->layers[l];
    const bool last = l == n->L - 1;
    const float* b = n->params + ly.b_off;
    hipError_t e;
    if (last && ly.wn) {
      const int blocks = (n->g.nx / lbmnn::kTX) * (n->g.ny / lbmnn::kTY) * (n->g.nz / lbmnn::kTZ);
      hipLaunchKernelGGL(lbmnn::conv_narrow_kernel, dim3(blocks), dim3(64 * lbmnn::kW), 0, n->stream, n->act[l], ly.wn,
                         b, yout, ly.cout, n->g, n->V);
      e = hipGetLastError();
    } else if (ly.wq) {
      const int blocks = (n->g.nx / lbmnn::kTX) * (n->g.ny / lbmnn::kTY) * (n->g.nz / lbmnn::kTZ);
      if (direct)
        hipLaunchKernelGGL((lbmnn::conv_pair_kernel<true>), dim3(blocks), dim3(64 * lbmnn::kW), 0, n->stream, nullptr,
                           x, n->ch[0], n->mean, n->inv_std, ly.wq, b, 1, n->act[l + 1], ly.cout, n->g, n->V);
      else
        hipLaunchKernelGGL((lbmnn::conv_pair_kernel<false>), dim3(blocks), dim3(64 * lbmnn::kW), 0, n->stream,
                           n->act[l], nullptr, 0, nullptr, nullptr, ly.wq, b, 1, n->act[l + 1], ly.cout, n->g, n->V);
      e = hipGetLastError();
    } else if (ly.cinp == 16)
      e = last ? conv<16, true>(n, n->act[l], ly.wp, b, 0, nullptr, yout, ly.cout)
               : conv<16, false>(n, n->act[l], ly.wp, b, 1, nullptr, n->act[l + 1], ly.cout);
    else
      e = last ? conv<32, true>(n, n->act[l], ly.wp, b, 0, nullptr, yout, ly.cout)
               : conv<32, false>(n, n->act[l], ly.wp, b, 1, nullptr, n->act[l + 1], ly.cout);
    NN_HIP(e, "conv forward");
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_nn_create(lbm_nn* out, int layers, const int* channels, const int64_t dims[3]) {
  if (!out) return nn_fail(LBM_EINVAL, "lbm_nn_create: out is NULL");
  *out = nullptr;
  if (layers < 1 || !channels || !dims) return nn_fail(LBM_EINVAL, "lbm_nn_create: bad layer description");
  if (channels[0] < 1 || channels[0] > 16) return nn_fail(LBM_EINVAL, "lbm_nn_create: input channels must be 1..16");
  for (int l = 1; l < layers; ++l)
    if (channels[l] != 32) return nn_fail(LBM_EINVAL, "lbm_nn_create: hidden widths must be 32");
  if (channels[layers] < 1 || channels[layers] > 32)
    return nn_fail(LBM_EINVAL, "lbm_nn_create: output channels must be 1..32");
  for (int a = 0; a < 3; ++a)
    if (dims[a] < 1 || dims[a] > 4096) return nn_fail(LBM_EINVAL, "lbm_nn_create: dims out of range");
  const int64_t V = dims[0] * dims[1] * dims[2];
  if (dims[0] % lbmnn::kTX || dims[1] % lbmnn::kTY || dims[2] % lbmnn::kTZ || V > (1 << 26))
    return nn_fail(LBM_EINVAL, "lbm_nn_create: nx must be a multiple of 32, ny and nz of 4 (at most 2^26 nodes)");
  lbm_nn n = new (std::nothrow) lbm_nn_ctx();
  if (!n) return nn_fail(LBM_ENOMEM, "lbm_nn_create: host allocation failed");
  n->L = layers;
  n->ch.assign(channels, channels + layers + 1);
  n->g = {(int)dims[0], (int)dims[1], (int)dims[2]};
  n->V = (int)V;
  long long off = 0;
  for (int l = 0; l < layers; ++l) {
    Layer ly;
    ly.cin = channels[l];
    ly.cout = channels[l + 1];
    ly.cinp = l == 0 ? 16 : 32;
    ly.w_off = off;
    off += 27LL * ly.cin * ly.cout;
    ly.b_off = off;
    off += ly.cout;
    n->layers.push_back(ly);
  }
  n->nparam = off;
  int rc = LBM_OK;
  auto alloc = [&](void** p, size_t bytes) {
    if (rc != LBM_OK) return;
    const hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) rc = nn_hip(e, "lbm_nn_create: hipMalloc");
  };
  hipError_t e0 = hipGetDevice(&n->device);
  if (e0 != hipSuccess) rc = nn_hip(e0, "hipGetDevice");
  const size_t P = sizeof(float) * (size_t)off;
  alloc((void**)&n->params, P);
  alloc((void**)&n->grads, P);
  alloc((void**)&n->m, P);
  alloc((void**)&n->v, P);
  alloc((void**)&n->mean, 16 * sizeof(float));
  alloc((void**)&n->inv_std, 16 * sizeof(float));
  alloc((void**)&n->out_std, 32 * sizeof(float));
  alloc((void**)&n->inv_out_std, 32 * sizeof(float));
  n->act.assign(layers, nullptr);
  for (int l = 0; l < layers; ++l) alloc((void**)&n->act[l], sizeof(__bf16) * (size_t)V * (l == 0 ? 16 : 32));
  alloc((void**)&n->dA, sizeof(__bf16) * (size_t)V * 32);
  alloc((void**)&n->dB, sizeof(__bf16) * (size_t)V * 32);
  alloc((void**)&n->y, sizeof(float) * (size_t)V * 32);
  alloc((void**)&n->part, sizeof(float) * 28 * (size_t)lbmnn::kGMaxBlocks * 1024);
  alloc((void**)&n->part2, sizeof(float) * 28 * (size_t)lbmnn::kGSegments * 1024);
  alloc((void**)&n->lpart, sizeof(double) * (size_t)((V + 255) / 256));
  alloc((void**)&n->loss_acc, sizeof(double));
  alloc((void**)&n->fld, sizeof(float) * 16 * (size_t)V);
  alloc((void**)&n->dfld, sizeof(double) * 10 * (size_t)V);
  for (int l = 0; l < layers; ++l) {
    Layer& ly = n->layers[l];
    alloc((void**)&ly.wp, sizeof(__bf16) * 27 * ly.cinp * 32);
    alloc((void**)&ly.wb, sizeof(__bf16) * 27 * 32 * 32);
    if (l == layers - 1 && ly.cinp == 32 && ly.cout <= 16) alloc((void**)&ly.wn, sizeof(__bf16) * 27 * 16 * 32);
    if (l == 0 && layers > 1 && ly.cin <= 8) alloc((void**)&ly.wq, sizeof(__bf16) * 14 * 32 * 16);
  }
  if (rc == LBM_OK) {
    std::vector<float> mean(16, 0.f), one(32, 1.f);
    hipError_t e = hipMemset(n->params, 0, P);
    if (e == hipSuccess) e = hipMemset(n->grads, 0, P);
    if (e == hipSuccess) e = hipMemset(n->m, 0, P);
    if (e == hipSuccess) e = hipMemset(n->v, 0, P);
    if (e == hipSuccess) e = hipMemset(n->loss_acc, 0, sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(n->mean, mean.data(), 16 * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(n->inv_std, one.data(), 16 * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(n->out_std, one.data(), 32 * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(n->inv_out_std, one.data(), 32 * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) rc = nn_hip(e, "lbm_nn_create: initialise");
  }
  if (rc == LBM_OK) rc = nn_pack_weights(n);
  if (rc == LBM_OK) {
    const hipError_t e = hipStreamSynchronize(n->stream);
    if (e != hipSuccess) rc = nn_hip(e, "hipStreamSynchronize");
  }
  if (rc != LBM_OK) {
    lbm_nn_destroy(n);
    return rc;
  }
  *out = n;
  return LBM_OK;
}

int lbm_nn_destroy(lbm_nn n) {
  if (!n) return LBM_OK;
  (void)nn_select(n);
  if (n->stream) (void)hipStreamSynchronize(n->stream);
  for (void* p : {(void*)n->params, (void*)n->grads, (void*)n->m, (void*)n->v, (void*)n->mean, (void*)n->inv_std,
                  (void*)n->out_std, (void*)n->inv_out_std, (void*)n->dA, (void*)n->dB, (void*)n->y, (void*)n->part, (void*)n->part2, (void*)n->lpart,
                  (void*)n->loss_acc, (void*)n->fld, (void*)n->dfld})
    if (p) (void)hipFree(p);
  for (__bf16* p : n->act)
    if (p) (void)hipFree(p);
  for (Layer& ly : n->layers) {
    if (ly.wp) (void)hipFree(ly.wp);
    if (ly.wb) (void)hipFree(ly.wb);
    if (ly.wn) (void)hipFree(ly.wn);
    if (ly.wq) (void)hipFree(ly.wq);
  }
  delete n;
  return LBM_OK;
}

int lbm_nn_set_stream(lbm_nn n, void* s) {
  if (!n) return nn_fail(LBM_EINVAL, "lbm_nn_set_stream: NULL network");
  n->stream = static_cast<hipStream_t>(s);
  return LBM_OK;
}

int64_t lbm_nn_param_count(lbm_nn n) { return n ? n->nparam : -1; }

int lbm_nn_set_params(lbm_nn n, const float* params, int mem) {
  if (!n || !params) return nn_fail(LBM_EINVAL, "lbm_nn_set_params: NULL argument");
  if (mem != LBM_HOST && mem != LBM_DEVICE) return nn_fail(LBM_EINVAL, "lbm_nn_set_params: bad memory kind");
  int rc = nn_select(n);
  if (rc) return rc;
  NN_HIP(hipMemcpyAsync(n->params, params, sizeof(float) * n->nparam,
                        mem == LBM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, n->stream),
         "copy params");
  if ((rc = nn_pack_weights(n))) return rc;
  NN_HIP(hipStreamSynchronize(n->stream), "hipStreamSynchronize");
  return LBM_OK;
}

static int nn_copy_out(lbm_nn n, float* dst, const float* src, int mem, const char* what) {
  if (!n || !dst) return nn_fail(LBM_EINVAL, std::string(what) + ": NULL argument");
  if (mem != LBM_HOST && mem != LBM_DEVICE) return nn_fail(LBM_EINVAL, std::string(what) + ": bad memory kind");
  int rc = nn_select(n);
  if (rc) return rc;
  NN_HIP(hipMemcpyAsync(dst, src, sizeof(float) * n->nparam,
                        mem == LBM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, n->stream),
         what);
  NN_HIP(hipStreamSynchronize(n->stream), "hipStreamSynchronize");
  return LBM_OK;
}

int lbm_nn_get_params(lbm_nn n, float* p, int mem) { return nn_copy_out(n, p, n ? n->params : nullptr, mem, "lbm_nn_get_params"); }
int lbm_nn_get_grads(lbm_nn n, float* g, int mem) { return nn_copy_out(n, g, n ? n->grads : nullptr, mem, "lbm_nn_get_grads"); }

int lbm_nn_zero_grad(lbm_nn n) {
  if (!n) return nn_fail(LBM_EINVAL, "lbm_nn_zero_grad: NULL network");
  int rc = nn_select(n);
  if (rc) return rc;
  NN_HIP(hipMemsetAsync(n->grads, 0, sizeof(float) * n->nparam, n->stream), "zero grads");
  return LBM_OK;
}

int lbm_nn_set_scaling(lbm_nn n, const double* mean, const double* sd, const double* out_sd) {
  if (!n || !mean || !sd) return nn_fail(LBM_EINVAL, "lbm_nn_set_scaling: NULL argument");
  std::vector<float> m(16, 0.f), is(16, 1.f), os(32, 1.f), ios(32, 1.f);
  for (int c = 0; c < n->ch[0]; ++c) {
    if (!(sd[c] > 0.0) || !std::isfinite(sd[c]) || !std::isfinite(mean[c]))
      return nn_fail(LBM_EINVAL, "lbm_nn_set_scaling: std must be finite and > 0");
    m[c] = (float)mean[c];
    is[c] = (float)(1.0 / sd[c]);
  }
  const double* o = out_sd ? out_sd : sd;
  for (int c = 0; c < n->ch[n->L]; ++c) {
    if (!(o[c] > 0.0) || !std::isfinite(o[c]))
      return nn_fail(LBM_EINVAL, "lbm_nn_set_scaling: out_std must be finite and > 0");
    os[c] = (float)o[c];
    ios[c] = (float)(1.0 / o[c]);
  }
  int rc = nn_select(n);
  if (rc) return rc;
  NN_HIP(hipMemcpyAsync(n->mean, m.data(), 16 * sizeof(float), hipMemcpyHostToDevice, n->stream), "copy mean");
  NN_HIP(hipMemcpyAsync(n->inv_std, is.data(), 16 * sizeof(float), hipMemcpyHostToDevice, n->stream), "copy std");
  NN_HIP(hipMemcpyAsync(n->out_std, os.data(), 32 * sizeof(float), hipMemcpyHostToDevice, n->stream), "copy out_std");
  NN_HIP(hipMemcpyAsync(n->inv_out_std, ios.data(), 32 * sizeof(float), hipMemcpyHostToDevice, n->stream),
         "copy out_std");
  NN_HIP(hipStreamSynchronize(n->stream), "hipStreamSynchronize");
  return LBM_OK;
}

int lbm_nn_set_output_offset(lbm_nn n, int offset) {
  if (!n) return nn_fail(LBM_EINVAL, "lbm_nn_set_output_offset: NULL network");
  if (offset < 0 || offset + n->ch[n->L] > n->ch[0])
    return nn_fail(LBM_EINVAL, "lbm_nn_set_output_offset: offset + output channels must not exceed the input channels");
  n->out_off = offset;
  return LBM_OK;
}

int lbm_nn_set_correction_limit(lbm_nn n, double limit) {
  if (!n) return nn_fail(LBM_EINVAL, "lbm_nn_set_correction_limit: NULL network");
  if (!(limit >= 0.0) || !std::isfinite(limit))
    return nn_fail(LBM_EINVAL, "lbm_nn_set_correction_limit: limit must be finite and >= 0");
  n->limit = limit;
  return LBM_OK;
}

int lbm_nn_forward(lbm_nn n, const float* x, float* y) {
  if (!n || !x || !y) return nn_fail(LBM_EINVAL, "lbm_nn_forward: NULL argument");
  int rc = nn_select(n);
  if (rc) return rc;
  // inference: the first layer reads x directly and the last writes y
  return nn_forward(n, x, y, false);
}

int lbm_nn_loss_backward(lbm_nn n, const float* x, const float* target, double* loss) {
  if (!n || !x || !target) return nn_fail(LBM_EINVAL, "lbm_nn_loss_backward: NULL argument");
  if (n->out_off + n->ch[n->L] > n->ch[0])
    return nn_fail(LBM_EINVAL, "lbm_nn_loss_backward: output fields beyond the input fields");
  int rc = nn_select(n);
  if (rc) return rc;
  if ((rc = nn_forward(n, x))) return rc;
  const int V = n->V, C = n->ch[n->L];
  const int lblocks = (V + 255) / 256;
  hipLaunchKernelGGL(lbmnn::loss_kernel, dim3(lblocks), dim3(256), 0, n->stream, n->y, x, target, n->inv_out_std, C,
                     n->out_off, V,
                     n->dA, n->lpart);
  NN_HIP(hipGetLastError(), "loss kernel");
  // dA holds the gradient with respect to the output of layer l (pre-ReLU for l < L-1)
  __bf16 *dcur = n->dA, *dnext = n->dB;
  const int ntiles = (n->g.nx / lbmnn::kGX) * (n->g.ny / lbmnn::kGY) * (n->g.nz / lbmnn::kGZ);
  const int tpb = (ntiles + lbmnn::kGMaxBlocks - 1) / lbmnn::kGMaxBlocks;
  const int nblk = (ntiles + tpb - 1) / tpb;
  for (int l = n->L - 1; l >= 0; --l) {
    const Layer& ly = n->layers[l];
    if (ly.cinp == 16)
      hipLaunchKernelGGL((lbmnn::wgrad_kernel<16>), dim3(nblk), dim3(256), 0, n->stream, n->act[l], dcur, n->part, n->g,
                         ntiles, tpb, ly.cin, ly.cout);
    else
      hipLaunchKernelGGL((lbmnn::wgrad_kernel<32>), dim3(nblk), dim3(256), 0, n->stream, n->act[l], dcur, n->part, n->g,
                         ntiles, tpb, ly.cin, ly.cout);
    NN_HIP(hipGetLastError(), "weight gradient kernel");
    const int nseg = nblk < lbmnn::kGSegments ? nblk : lbmnn::kGSegments;
    const int cio = ly.cin * ly.cout, sum_blocks = (28 * cio + 255) / 256;
    hipLaunchKernelGGL(lbmnn::wgrad_partial_sum_kernel, dim3(sum_blocks, nseg), dim3(256), 0, n->stream, n->part,
                       nblk, nseg, cio, n->part2);
    NN_HIP(hipGetLastError(), "weight gradient partial sums");
    hipLaunchKernelGGL(lbmnn::wgrad_reduce_kernel, dim3(sum_blocks), dim3(256), 0, n->stream, n->part2, nseg,
                       ly.cin, ly.cout, n->grads + ly.w_off, n->grads + ly.b_off);
    NN_HIP(hipGetLastError(), "weight gradient reduction");
    if (l > 0) {
      // gradient with respect to this layer's input = previous output; times the ReLU derivative
      NN_HIP((conv<32, false>(n, dcur, ly.wb, nullptr, 0, n->act[l], dnext, 32)), "conv backward-data");
      __bf16* t = dcur;
      dcur = dnext;
      dnext = t;
    }
  }
  if (loss) {
    std::vector<double> h(lblocks);
    NN_HIP(hipMemcpyAsync(h.data(), n->lpart, sizeof(double) * lblocks, hipMemcpyDeviceToHost, n->stream),
           "copy loss");
    NN_HIP(hipStreamSynchronize(n->stream), "hipStreamSynchronize");
    double s = 0.0;
    for (double x2 : h) s += x2;
    *loss = s / ((double)C * V);
  } else {
    hipLaunchKernelGGL(lbmnn::loss_accumulate_kernel, dim3(1), dim3(256), 0, n->stream, n->lpart, lblocks,
                       1.0 / ((double)C * V), n->loss_acc);
    NN_HIP(hipGetLastError(), "loss accumulation");
    ++n->loss_count;
  }
  return LBM_OK;
}

int lbm_nn_take_loss(lbm_nn n, double* sum, int64_t* count) {
  if (!n || !sum) return nn_fail(LBM_EINVAL, "lbm_nn_take_loss: NULL argument");
  int rc = nn_select(n);
  if (rc) return rc;
  NN_HIP(hipMemcpyAsync(sum, n->loss_acc, sizeof(double), hipMemcpyDeviceToHost, n->stream), "copy loss sum");
  NN_HIP(hipMemsetAsync(n->loss_acc, 0, sizeof(double), n->stream), "reset loss sum");
  NN_HIP(hipStreamSynchronize(n->stream), "hipStreamSynchronize");
  if (count) *count = n->loss_count;
  n->loss_count = 0;
  return LBM_OK;
}

int lbm_nn_adam_step(lbm_nn n, double lr, double beta1, double beta2, double eps, double grad_scale, int64_t t) {
  if (!n) return nn_fail(LBM_EINVAL, "lbm_nn_adam_step: NULL network");
  if (t < 1 || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
    return nn_fail(LBM_EINVAL, "lbm_nn_adam_step: bad hyper-parameters");
  int rc = nn_select(n);
  if (rc) return rc;
  const float c1 = (float)(1.0 / (1.0 - std::pow(beta1, (double)t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(beta2, (double)t)));
  hipLaunchKernelGGL(lbmnn::adam_kernel, dim3((unsigned)((n->nparam + 255) / 256)), dim3(256), 0, n->stream,
                     n->params, n->grads, n->m, n->v, n->nparam, (float)lr, (float)beta1, (float)beta2, (float)eps,
                     (float)grad_scale, c1, c2);
  NN_HIP(hipGetLastError(), "adam kernel");
  return nn_pack_weights(n);
}

int lbm_nn_fields_to_planes(int D, int64_t nodes, const double* rho, const double* u, const double* T, float* x,
                            void* stream) {
  if (!rho || !u || !T || !x) return nn_fail(LBM_EINVAL, "lbm_nn_fields_to_planes: NULL argument");
  if ((D != 2 && D != 3) || nodes < 1 || nodes > (1LL << 31) - 256)
    return nn_fail(LBM_EINVAL, "lbm_nn_fields_to_planes: bad lattice or node count");
  const int V = (int)nodes;
  hipLaunchKernelGGL(lbmnn::fields_to_input_kernel, dim3((V + 255) / 256), dim3(256), 0,
                     static_cast<hipStream_t>(stream), rho, u, T, D, V, x);
  NN_HIP(hipGetLastError(), "fields kernel");
  return LBM_OK;
}

int lbm_nn_correct(lbm_nn n, lbm_handle h) {
  if (!n || !h) return nn_fail(LBM_EINVAL, "lbm_nn_correct: NULL argument");
  const int D = h->lattice;
  if (n->ch[0] != D + 2 || n->out_off + n->ch[n->L] > D + 2)
    return nn_fail(LBM_EINVAL, "lbm_nn_correct: the network must read the D + 2 fields and correct fields among them");
  if (h->n[0] != n->g.nx || h->n[1] != n->g.ny || h->n[2] != n->g.nz)
    return nn_fail(LBM_EINVAL, "lbm_nn_correct: grid of the handle differs from the network's");
  int rc = nn_select(n);
  if (rc) return rc;
  const int V = n->V;
  double* drho = n->dfld;
  double* du = drho + V;
  double* dT = du + 3 * (size_t)V;
  // everything on the handle's stream: moments, network, increments
  hipStream_t saved = n->stream;
  n->stream = h->stream;
  if ((rc = lbm::fields_current(h)) == LBM_OK) {
    const double* F = h->fields;  // rho, u_x, u_y, u_z, T, rho E planes
    hipLaunchKernelGGL(lbmnn::fields_to_input_kernel, dim3((V + 255) / 256), dim3(256), 0, n->stream, F, F + V,
                       F + 4 * (size_t)V, D, V, n->fld);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) rc = nn_hip(e, "fields kernel");
    if (rc == LBM_OK) rc = nn_forward(n, n->fld, nullptr, false);
    if (rc == LBM_OK) {
      hipLaunchKernelGGL(lbmnn::output_to_increments_kernel, dim3((V + 255) / 256), dim3(256), 0, n->stream, n->y,
                         n->out_std, n->ch[n->L], n->out_off, D, (float)n->limit, V, drho, du, dT);
      e = hipGetLastError();
      if (e != hipSuccess) rc = nn_hip(e, "increments kernel");
    }
    if (rc == LBM_OK) rc = lbm::fields_increment_async(h, drho, du, dT);
  }
  n->stream = saved;
  return rc;
}

}  // extern "C"
