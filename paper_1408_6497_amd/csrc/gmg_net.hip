// Learned smoother kernels: a 3-layer 3x3x3 convolutional net on the DoF
// lattice of one level (circular padding, no bias, 16 hidden channels), its
// backward pass and an Adam step.
//
//   x_in = bf16(D^-1 r / s)                       s = RMS(D^-1 r)
//   a1   = bf16(relu(W1 * x_in))                  1 -> 16 channels
//   a2   = bf16(relu(W2 * a1))                    16 -> 16 (MFMA)
//   y    = W3 * a2                                16 -> 1
//   u   += s y                                    (learned correction)
//
// Weights and activations are BF16 (round to nearest even from FP32), every
// accumulation is FP32.  Activations are channels-last: 16 BF16 values (32
// bytes) per voxel, voxel index i + N (j + N k).  A tap t = (dz+1) 9 + (dy+1) 3
// + (dx+1) reads the voxel at offset (dx, dy, dz), wrapped periodically.
//
// Forward pass, two kernels per application:
//   k_net_l12  one 16x8x4 brick per block: bf16(x) with a two-voxel halo in LDS,
//              expanded into x-triples (the three dx taps of a row in 8 bytes);
//              layer 1 on the matrix cores over the brick plus a one-voxel halo
//              (9 rows of 3 taps as K = 36 of 64: two v_mfma_f32_16x16x32_bf16 per 16
//              voxels); a1 stays in LDS; layer 2 (6912 of the 7776 multiply-adds per voxel) on
//              v_mfma_f32_16x16x32_bf16 with two (dz, dx) offsets of one input row per
//              B operand (16 voxels along x, 8 channels per lane) and the matching
//              16 x 32 weight blocks as A (registers), accumulating 16 output channels
//              x 16 voxels; a2 to HBM (32 B per voxel), a1 only when training keeps it.
//   k_net_l3s  layer 3 streamed along z over 16x16 output columns (lattices of 128 nodes
//              and more; k_net_l3m on the bricks below that): per row of each a2 plane the
//              nine (dz, dy) partial sums over dx and channels on the MFMA (fixed A), then
//              three rolling output planes, with u += s y fused.
// The backward-data pass of layer 2 (k_net_l2bwd) runs the same MFMA loop with the
// flipped, transposed weights and the ReLU mask of the forward pass.
#include <algorithm>

#include "gmg_kernels.h"

namespace gmg {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int kNC = 16;
constexpr int kTaps = 27;
constexpr int kBlk = 256;

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two FP32 values to packed BF16 (round to nearest even: v_cvt_pk_bf16_f32), a in the low half.
typedef float float2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(float2v{a, b}, bf16x2));
}

typedef short short2v __attribute__((ext_vector_type(2)));

// bf16(relu(a)), bf16(relu(b)) packed, a in the low half: rounded first, then every value with
// the sign bit set (negative or -0) cleared by a 16-bit integer max with 0 (v_pk_max_i16).
// Rounding to nearest keeps the sign, so this equals rounding the rectified values.
__device__ __forceinline__ uint32_t pack2_relu(float a, float b) {
  const short2v v = __builtin_bit_cast(short2v, pack2(a, b));
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(v, short2v{0, 0}));
}

__device__ __forceinline__ size_t vox(int i, int j, int k, int N) {
  return (static_cast<size_t>(k) * N + j) * N + i;
}

// voxel index of (i, j, k) + offset of tap t (sign +1) or - offset (sign -1)
__device__ __forceinline__ size_t nbr(int i, int j, int k, int t, int sign, int N) {
  const int m = N - 1;
  const int dx = (t % 3) - 1, dy = ((t / 3) % 3) - 1, dz = (t / 9) - 1;
  return vox((i + sign * dx) & m, (j + sign * dy) & m, (k + sign * dz) & m, N);
}

struct ClassTab64 {
  double v[64];
};

// ---------------------------------------------------------------------------- input
// x_in = bf16(D^-1 r / s) with s = sqrt(ssum / N^3) (or x_in = bf16(x) when dinv is null);
// four consecutive voxels of a row per thread (N is a multiple of 4), s formed once per thread.
constexpr int kInThreads = 64;

__global__ void __launch_bounds__(kInThreads) k_net_in(const float* __restrict__ r, const ClassTab64 dinv,
                                                       const int q, const int use_dinv,
                                                       const double* __restrict__ ssum, const int N,
                                                       uint16_t* __restrict__ xin) {
  const int i0 = 4 * (blockIdx.x * kInThreads + threadIdx.x);
  const int j = blockIdx.y, k = blockIdx.z;
  if (i0 >= N) return;
  const size_t v = vox(i0, j, k, N);
  const float4 x4 = *reinterpret_cast<const float4*>(r + v);
  float x[4] = {x4.x, x4.y, x4.z, x4.w};
  if (use_dinv) {
    const double nn = static_cast<double>(N) * N * N;
    const float s = static_cast<float>(sqrt(*ssum / nn));
    const int base = q * ((j % q) + q * (k % q));
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float d = static_cast<float>(dinv.v[base + (i0 + e) % q]);
      x[e] = (s > 0.0f) ? (d * x[e]) / s : 0.0f;
    }
  }
  *reinterpret_cast<u32x2*>(xin + v) = u32x2{pack2(x[0], x[1]), pack2(x[2], x[3])};
}

// sum over voxels of (D^-1 r)^2, one partial per (j, k) row; four consecutive voxels per thread
__global__ void __launch_bounds__(kBlk) k_net_sqsum(const float* __restrict__ r, const ClassTab64 dinv, const int q,
                                                    const int N, double* part) {
  __shared__ double red[kBlk / 64];
  const int j = blockIdx.y, k = blockIdx.z;
  double s = 0.0;
  const float* row = r + (static_cast<size_t>(k) * N + j) * N;
  const int base = q * ((j % q) + q * (k % q));
  for (int i0 = 4 * threadIdx.x; i0 < N; i0 += 4 * blockDim.x) {
    const float4 x4 = *reinterpret_cast<const float4*>(row + i0);
    const float x[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float d = static_cast<float>(dinv.v[base + (i0 + e) % q]);
      const double t = static_cast<double>(d * x[e]);
      s = fma(t, t, s);
    }
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < static_cast<int>(blockDim.x / 64); ++w) t += red[w];
    part[static_cast<size_t>(k) * N + j] = t;
  }
}

// ---------------------------------------------------------------------------- layer 2 (16 -> 16, MFMA)
// Bricks of 16x8x4 output voxels; one block of four wavefronts per brick, wavefront tz owning
// the 8 output rows (16 voxels along x each) of plane tz.  The 16-channel input of the brick
// plus a one-voxel halo sits in LDS as two half tiles (channels 0-7 and 8-15, 16 bytes per
// voxel each), so the 16-byte reads of 16 consecutive voxels are free of bank conflicts.
//
// The contraction over 27 taps x 16 input channels runs on v_mfma_f32_16x16x32_bf16 (K = 32):
// the 9 (dz, dx) offsets are taken in pairs (the last with an empty partner), so one B operand
// holds one input row (16 voxels, 8 channels per lane) at two offsets, and the A operand the
// matching 16 x 32 weight block for one dy.  Every row loaded from LDS feeds the up to three
// output rows it is a y-neighbour of: 50 B loads and 120 MFMAs per wavefront.
constexpr int kBX = 16, kBY = 8, kBZ = 4;
constexpr int kHX = kBX + 2, kHY = kBY + 2, kHZ = kBZ + 2;
constexpr int kHalo = kHX * kHY * kHZ;  // 1080 voxels
constexpr int kHalf = kHalo + 4;        // half-tile stride in 16-byte entries (bank offset 16)
constexpr int kPairs = 5;               // ceil(9 / 2) (dz, dx) pairs


__device__ __forceinline__ floatx4 mfma32(const u32x4 a, const u32x4 b, const floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

// Brick of this block.  Blocks go to the XCDs round-robin (blockIdx mod 8), so block b is taken
// as the (b / 8)-th brick of XCD b mod 8, and each XCD owns a contiguous range of bricks in an
// order with z fastest, then x, then y: the bricks a XCD has in flight at once are mostly z
// neighbours and share their halo planes in that XCD's L2.  The brick count (N / 16)(N / 8)(N / 4)
// is a multiple of 8 for N >= 16.
__device__ __forceinline__ void brick_of(int N, int& x0, int& y0, int& z0) {
  const int nbx = N / kBX, nbz = N / kBZ;
  const int per_xcd = (nbx * (N / kBY) * nbz) >> 3;
  const int l = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  z0 = (l % nbz) * kBZ;
  x0 = ((l / nbz) % nbx) * kBX;
  y0 = (l / (nbz * nbx)) * kBY;
}

// (dz, dx) offset of slot f (0, 1) of pair p; the empty partner of the last pair repeats
// offset 8 (its weights are zero)
__device__ __forceinline__ int pair_combo(int p, int f) { return min(2 * p + f, 8); }

// A operands of layer 2 for this lane from the lane-ordered copy k_net_pack_lanes writes:
// entry (p, dy) of lane l is W[t][l & 15][8h .. 8h + 7] for the tap t of pair p, slot g >> 1, dy
// (g = l >> 4, h = g & 1), zero for the empty slot -- one 16-byte load per operand.
__device__ __forceinline__ void load_l2_weights(const u32x4* __restrict__ wl, int lane, u32x4 (&wa)[kPairs][3]) {
#pragma unroll
  for (int p = 0; p < kPairs; ++p)
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) wa[p][dy] = wl[(p * 3 + dy) * 64 + lane];
}

// acc[ty] (output channels 4g .. 4g+3 of voxel (col, ty, tz)) = sum over taps and input channels.
// The five B operands of input row r + 1 are loaded while the MFMAs of row r run.
__device__ __forceinline__ void layer2_wave(const u32x4* __restrict__ tile, const u32x4 (&wa)[kPairs][3], int tz,
                                            int col, int g, floatx4 (&acc)[kBY]) {
  const int h = g & 1;
#pragma unroll
  for (int ty = 0; ty < kBY; ++ty) acc[ty] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  // per pair: this lane's offset into the tile (slot g >> 1)
  int off[kPairs];
#pragma unroll
  for (int p = 0; p < kPairs; ++p) {
    const int c = pair_combo(p, g >> 1);
    const int dz = c / 3 - 1, dx = c % 3 - 1;
    off[p] = h * kHalf + ((tz + 1 + dz) * kHY) * kHX + (col + 1 + dx);
  }
  u32x4 bq[2][kPairs];
#pragma unroll
  for (int p = 0; p < kPairs; ++p) bq[0][p] = tile[off[p]];
#pragma unroll
  for (int r = 0; r < kHY; ++r) {
    if (r + 1 < kHY) {
#pragma unroll
      for (int p = 0; p < kPairs; ++p) bq[(r + 1) & 1][p] = tile[off[p] + (r + 1) * kHX];
    }
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const int ty = r - dy;  // the row whose tap dy - 1 reads row r
        if (ty < 0 || ty >= kBY) continue;
        acc[ty] = mfma32(wa[p][dy], bq[r & 1][p], acc[ty]);
      }
    }
    __builtin_amdgcn_iglp_opt(0);
  }
}

// The 16-channel input of a brick plus a one-voxel halo (kHX x kHY x kHZ voxels, periodic wrap)
// into the two half tiles, plane by plane: thread t takes the half-voxel entries t and t + 256 of
// every plane (360 per plane), so the row and column part of each global address is formed once
// and all loads are issued before the first LDS store.
__device__ __forceinline__ void fill_halo_tile(const u32x4* __restrict__ in4, int N, int x0, int y0, int z0,
                                               u32x4* __restrict__ tile) {
  constexpr int kPlane = kHX * kHY * 2;  // 360 half-voxel entries per plane
  const int m = N - 1;
  int src[2], dst[2];
  bool use[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int e = threadIdx.x + k * kBlk;
    use[k] = e < kPlane;
    const int ee = use[k] ? e : 0;
    const int h = ee & 1, vx = ee >> 1;
    const int hx = vx % kHX, hy = vx / kHX;
    src[k] = ((((y0 - 1 + hy) & m) * N + ((x0 - 1 + hx) & m)) << 1) + h;
    dst[k] = h * kHalf + hy * kHX + hx;
  }
  u32x4 v[kHZ][2];
#pragma unroll
  for (int hz = 0; hz < kHZ; ++hz) {
    const size_t zoff = static_cast<size_t>((z0 - 1 + hz) & m) * N * N * 2;
#pragma unroll
    for (int k = 0; k < 2; ++k)
      if (use[k]) v[hz][k] = in4[zoff + src[k]];
  }
#pragma unroll
  for (int hz = 0; hz < kHZ; ++hz)
#pragma unroll
    for (int k = 0; k < 2; ++k)
      if (use[k]) tile[dst[k] + hz * kHX * kHY] = v[hz][k];
}

// out[v][m] = sum_t sum_k wA[t][m][k] in[v + off(t)][k];  backward-data: bf16(. * 1[mask[v][m] > 0]).
// N >= 16.
__global__ void __launch_bounds__(kBlk) k_net_l2bwd(const uint16_t* __restrict__ in, const u32x4* __restrict__ wl,
                                                    const uint16_t* __restrict__ mask, const int N,
                                                    uint16_t* __restrict__ out) {
  __shared__ u32x4 tile[2 * kHalf];
  int x0, y0, z0;
  brick_of(N, x0, y0, z0);
  fill_halo_tile(reinterpret_cast<const u32x4*>(in), N, x0, y0, z0, tile);
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, g = lane >> 4;
  u32x4 wa[kPairs][3];
  load_l2_weights(wl, lane, wa);
  __syncthreads();
  const int tz = threadIdx.x >> 6;
  floatx4 acc[kBY];
  layer2_wave(tile, wa, tz, col, g, acc);
#pragma unroll
  for (int ty = 0; ty < kBY; ++ty) {
    const size_t v = vox(x0 + col, y0 + ty, z0 + tz, N);
    const u32x2 mk = reinterpret_cast<const u32x2*>(mask)[v * 4 + g];
    const float o0 = __uint_as_float(mk.x << 16) > 0.0f ? acc[ty][0] : 0.0f;
    const float o1 = __uint_as_float(mk.x & 0xFFFF0000u) > 0.0f ? acc[ty][1] : 0.0f;
    const float o2 = __uint_as_float(mk.y << 16) > 0.0f ? acc[ty][2] : 0.0f;
    const float o3 = __uint_as_float(mk.y & 0xFFFF0000u) > 0.0f ? acc[ty][3] : 0.0f;
    reinterpret_cast<u32x2*>(out)[v * 4 + g] = u32x2{pack2(o0, o1), pack2(o2, o3)};
  }
}

// ---------------------------------------------------------------------------- fused layers 1 + 2
// One block per 16x8x4 output brick.  bf16(x) of the brick plus a two-voxel halo goes to LDS and
// is expanded into x-triples: entry (c, row, plane) holds the inputs at columns c - 1, c, c + 1
// (and a zero), 8 bytes.  Layer 1 runs on the matrix cores over the brick plus a one-voxel halo,
// 16 voxels per step: the 27 taps are 9 (dz, dy) rows of 3 dx taps, each row one 8-byte read of
// a triple (4 K slots, the fourth with a zero weight); one v_mfma_f32_16x16x32_bf16 takes rows
// 0-7 (two per lane group) and a second one row 8.  ReLU and BF16 rounding into the half tiles
// layer 2 reads; layer 2 as above.  a1 never goes to HBM unless the caller keeps it (training:
// the backward pass reads it).
constexpr int kXX = kBX + 4, kXY = kBY + 4, kXZ = kBZ + 4;  // input tile with a two-voxel halo
constexpr int kTX = kBX + 2;                                 // triple columns (the layer-1 halo width)
constexpr int kTriples = kTX * kXY * kXZ;                    // 1728 entries of 8 bytes

template <bool KEEP_A1>
__global__ void __launch_bounds__(kBlk) k_net_l12(const uint16_t* __restrict__ xin, const u32x4* __restrict__ w1l,
                                                  const u32x4* __restrict__ wl, const int N,
                                                  uint16_t* __restrict__ a1_out, uint16_t* __restrict__ a2_out) {
  __shared__ u32x2 x3[kTriples];
  __shared__ u32x4 tile[2 * kHalf];
  static_assert(kXZ * kXY * kXX * sizeof(uint16_t) <= sizeof(tile), "the plain input tile fits in the half tiles");
  uint16_t* xt = reinterpret_cast<uint16_t*>(tile);  // plain input tile, dead once the triples are built
  int x0, y0, z0;
  brick_of(N, x0, y0, z0);
  const int m = N - 1;
  {  // plane by plane: thread t < 240 takes column t % 20 of row t / 20 in every plane, so the row
     // and column part of the global address is formed once; all loads before the first store
    constexpr int kRowCol = kXY * kXX;  // 240
    const int t = threadIdx.x < kRowCol ? threadIdx.x : 0;
    const int hx = t % kXX, hy = t / kXX;
    const int src = ((y0 - 2 + hy) & m) * N + ((x0 - 2 + hx) & m);
    uint16_t v[kXZ];
#pragma unroll
    for (int hz = 0; hz < kXZ; ++hz)
      v[hz] = xin[static_cast<size_t>((z0 - 2 + hz) & m) * N * N + src];
    if (threadIdx.x < kRowCol) {
#pragma unroll
      for (int hz = 0; hz < kXZ; ++hz) xt[hz * kRowCol + t] = v[hz];
    }
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 15;
  const int g = lane >> 4;
  // W1 as the A operands (lane-ordered copy, k_net_pack_lanes): row = output channel col; first
  // MFMA, lane group g: (dz, dy) rows 2g and 2g + 1, taps dx = -1, 0, 1 and a zero each; second
  // MFMA: row 8 in group 0, zeros elsewhere.  Tap of row rho and dx: 3 rho + dx + 1.
  const u32x4 w1a = w1l[lane], w1b = w1l[64 + lane];
  u32x4 wa[kPairs][3];
  load_l2_weights(wl, lane, wa);
  // this lane's triple offsets for rows 2g and 2g + 1 ((dz, dy) of row rho: rho / 3 - 1, rho % 3 - 1)
  const int offa = ((2 * g) / 3 - 1) * kXY * kTX + ((2 * g) % 3 - 1) * kTX;
  const int offb = ((2 * g + 1) / 3 - 1) * kXY * kTX + ((2 * g + 1) % 3 - 1) * kTX;
  constexpr int off8 = kXY * kTX + kTX;  // row 8: dz = dy = 1
  __syncthreads();
  // triples: entry (c - 1, row, plane) for triple columns c = 1 .. kTX of the input tile; thread
  // t < 216 takes column t % 18 of row t / 18 in every plane (constant offsets per plane)
  if (threadIdx.x < kTX * kXY) {
    const int c = threadIdx.x % kTX, row = threadIdx.x / kTX;
#pragma unroll
    for (int pl = 0; pl < kXZ; ++pl) {
      const uint16_t* src = xt + (pl * kXY + row) * kXX + c;
      x3[(pl * kXY + row) * kTX + c] = u32x2{static_cast<uint32_t>(src[0]) | (static_cast<uint32_t>(src[1]) << 16), src[2]};
    }
  }
  __syncthreads();
  // layer 1 over the 1080 voxels of the brick plus a one-voxel halo, 16 at a time: wavefront w
  // takes groups w, w + 4, ..., 17 of them (the last partly beyond the 1080).  Voxel e = hx + 18 hy
  // + 180 hz has its centre triple at e + 234 + 36 hz.
  constexpr int kGroups = (kHalo + 15) / 16;
  static_assert(kGroups % (kBlk / 64) == 0, "every wavefront takes the same number of groups");
  static_assert(kTX == kHX && kTX * (kXY - kHY) == 36 && kXY * kTX + kTX == 234, "triple index of a halo voxel");
  int e = 16 * wave + col;
  int hz = e / (kHX * kHY);
  int rem = e - hz * (kHX * kHY);
#pragma unroll
  for (int it = 0; it < kGroups / (kBlk / 64); ++it) {
    const bool live = e < kHalo;
    const int c3 = live ? e + off8 + 36 * hz : off8;  // centre triple of voxel e
    const u32x2 ta = x3[c3 + offa], tb = x3[c3 + offb], t8 = x3[c3 + off8];
    floatx4 acc = mfma32(w1a, u32x4{ta.x, ta.y, tb.x, tb.y}, floatx4{0.0f, 0.0f, 0.0f, 0.0f});
    acc = mfma32(w1b, u32x4{t8.x, t8.y, 0u, 0u}, acc);
    // lane holds output channels 4 g .. 4 g + 3 of voxel e: half g >> 1, bytes 8 (g & 1) ..
    const u32x2 pk{pack2_relu(acc[0], acc[1]), pack2_relu(acc[2], acc[3])};
    // lanes past the 1080 voxels store into the half tiles' padding (no branch in the loop)
    reinterpret_cast<u32x2*>(tile + (g >> 1) * kHalf + (live ? e : kHalo + (e & 3)))[g & 1] = pk;
    if (KEEP_A1 && live) {
      const int hy = rem / kHX, hx = rem - (rem / kHX) * kHX;
      if (hx >= 1 && hx <= kBX && hy >= 1 && hy <= kBY && hz >= 1 && hz <= kBZ)
        reinterpret_cast<u32x2*>(a1_out)[vox(x0 + hx - 1, y0 + hy - 1, z0 + hz - 1, N) * 4 + g] = pk;
    }
    e += 64;
    rem += 64;
    if (rem >= kHX * kHY) {
      rem -= kHX * kHY;
      ++hz;
    }
    __builtin_amdgcn_iglp_opt(0);
  }
  __syncthreads();
  static_assert(kBlk / 64 == kBZ, "one wave per plane of the brick");
  const int tz = wave;
  floatx4 acc[kBY];
  layer2_wave(tile, wa, tz, col, g, acc);
  u32x2* dst = reinterpret_cast<u32x2*>(a2_out) + vox(x0 + col, y0, z0 + tz, N) * 4 + g;
#pragma unroll
  for (int ty = 0; ty < kBY; ++ty)
    dst[static_cast<size_t>(ty) * N * 4] =
        u32x2{pack2_relu(acc[ty][0], acc[ty][1]), pack2_relu(acc[ty][2], acc[ty][3])};
}

// ---------------------------------------------------------------------------- layer 3 (16 -> 1, MFMA)
// y = W3 * a2, streamed along z: a block owns a 16x16 column of outputs and a segment of its
// planes, and walks the input planes once (segment plus one plane each side):
//   1. the plane of a2 with a one-voxel x and y halo (18x18 voxels) goes to LDS as two half
//      tiles; for each of its 18 rows the nine partial sums P[(dz, dy)](v) = sum_dx sum_c
//      W3[(dz, dy, dx)][c] a2[v + dx][c] come out of two v_mfma_f32_16x16x32_bf16 with a fixed
//      A: row m = 4 (dz + 1) + (dy + 1) holds the weights of (dz, dy) (rows 3, 7, 11 and 12-15
//      zero), K = (two dx offsets, 16 channels), then (dx = +1, zero); the B operands are the
//      row at dx = -1, 0 and +1;
//   2. the partial sums go to LDS (12 bytes per (row, dz, voxel)); thread (x, y) adds the three
//      dy values of each dz to the output plane that dz reaches (z - dz): plane p feeds outputs
//      p + 1, p and p - 1, kept in three rolling registers, and output p - 1 is complete and
//      stored (y = sum or y += s sum) after plane p.
// Each input plane is read once per column (a2 traffic 1.27x for the x and y halo, plus two planes
// per segment), where bricks with a z halo read it 2.1x; the next plane's loads are in flight
// while the current one is computed.
constexpr int kSX = 16, kSY = 16;               // output cross-section of a column
constexpr int kSHX = kSX + 2, kSHY = kSY + 2;   // with the halo
constexpr int kSHalf = kSHX * kSHY + 8;         // half-tile stride in 16-byte entries
constexpr int kSPlane = kSHX * kSHY * 2;        // 648 half-voxel entries per plane
constexpr int kSLoads = (kSPlane + kBlk - 1) / kBlk;  // 3 per thread
constexpr int kSRowsPerWave = (kSHY + 3) / 4;   // 5 (waves 2 and 3 take 4)
static_assert(kSX * kSY == kBlk, "one output per thread and plane");

__global__ void __launch_bounds__(kBlk) k_net_l3s(const uint16_t* __restrict__ a2, const u32x4* __restrict__ w3l,
                                                  const int N, const int nseg, const int mode,
                                                  const double* __restrict__ ssum, float* __restrict__ y) {
  __shared__ u32x4 abuf[2 * kSHalf];
  __shared__ float pbuf[kSHY * 3 * kSX * 3];  // [row][dz][x][dy]
  const int ncx = N / kSX, ncy = N / kSY;
  const int c = blockIdx.x % (ncx * ncy), seg = blockIdx.x / (ncx * ncy);
  const int x0 = (c % ncx) * kSX, y0 = (c / ncx) * kSY;
  const int L = N / nseg, zs = seg * L, ze = zs + L;
  const int m = N - 1;
  const u32x4* in4 = reinterpret_cast<const u32x4*>(a2);
  // this thread's half-voxel entries of every plane: row/column part of the address, LDS slot
  int src[kSLoads], dst[kSLoads];
  bool use[kSLoads];
#pragma unroll
  for (int k = 0; k < kSLoads; ++k) {
    const int e = threadIdx.x + k * kBlk;
    use[k] = e < kSPlane;
    const int ee = use[k] ? e : 0;
    const int h = ee & 1, vx = ee >> 1;
    const int hx = vx % kSHX, hy = vx / kSHX;
    src[k] = ((((y0 - 1 + hy) & m) * N + ((x0 - 1 + hx) & m)) << 1) + h;
    dst[k] = h * kSHalf + vx;
  }
  auto load_plane = [&](int p, u32x4 (&v)[kSLoads]) {
    const size_t zoff = static_cast<size_t>(p & m) * N * N * 2;
#pragma unroll
    for (int k = 0; k < kSLoads; ++k)
      if (use[k]) v[k] = in4[zoff + src[k]];
  };
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 15, g = lane >> 4;
  const u32x4 wA1 = w3l[lane], wA2 = w3l[64 + lane];
  const u32x4* t1 = abuf + (g & 1) * kSHalf + col + (g >> 1);
  const u32x4* t2 = abuf + (g & 1) * kSHalf + col + 2;
  const int ox = threadIdx.x & 15, oy = threadIdx.x >> 4;  // this thread's output column
  float sc = 1.0f;
  if (mode != 0) sc = static_cast<float>(sqrt(*ssum / (static_cast<double>(N) * N * N)));
  float a_prev = 0.0f, a_cur = 0.0f, a_next = 0.0f;  // outputs p - 1, p, p + 1
  u32x4 pre[kSLoads];
  load_plane(zs - 1, pre);
  for (int p = zs - 1; p <= ze; ++p) {
#pragma unroll
    for (int k = 0; k < kSLoads; ++k)
      if (use[k]) abuf[dst[k]] = pre[k];
    __syncthreads();
    if (p < ze) load_plane(p + 1, pre);
    floatx4 pr[kSRowsPerWave];
#pragma unroll
    for (int k = 0; k < kSRowsPerWave; ++k) {
      const int hy = wave + 4 * k;
      if (hy < kSHY) {
        pr[k] = mfma32(wA1, t1[hy * kSHX], floatx4{0.0f, 0.0f, 0.0f, 0.0f});
        pr[k] = mfma32(wA2, t2[hy * kSHX], pr[k]);
      }
    }
    if (g < 3) {
#pragma unroll
      for (int k = 0; k < kSRowsPerWave; ++k) {
        const int hy = wave + 4 * k;
        if (hy < kSHY) {
          float* d = pbuf + ((hy * 3 + g) * kSX + col) * 3;
          d[0] = pr[k][0];
          d[1] = pr[k][1];
          d[2] = pr[k][2];
        }
      }
    }
    __syncthreads();
    // dz index d reaches output p + 1 - d
    float sd[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      float t = 0.0f;
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) t += pbuf[(((oy + dy) * 3 + d) * kSX + ox) * 3 + dy];
      sd[d] = t;
    }
    a_next += sd[0];
    a_cur += sd[1];
    a_prev += sd[2];
    const int o = p - 1;  // complete now
    if (o >= zs && o < ze) {
      float* dsty = y + vox(x0 + ox, y0 + oy, o, N);
      if (mode == 0) *dsty = a_prev;
      else *dsty += sc * a_prev;
    }
    a_prev = a_cur;
    a_cur = a_next;
    a_next = 0.0f;
  }
}

// Layer 3 on the bricks of k_net_l12 (lattices below 128 nodes, where a z stream of a few planes
// per column would be latency-bound), in two stages:
//   1. for every row (hy, hz) of the brick plus a one-voxel halo (60 rows of 16 voxels) the
//      9 partial sums P[(dz, dy)](v) = sum_dx sum_c W3[(dz, dy, dx)][c] a2[v + dx][c] come out of
//      two v_mfma_f32_16x16x32_bf16 with a fixed A: row m = 4 (dz + 1) + (dy + 1) of A holds the
//      weights of (dz, dy) (rows 3, 7, 11 and 12-15 zero), K = (two dx offsets, 16 channels)
//      and (dx = +1, zero); the B operands are the a2 row at dx = -1, 0 and +1 from the half
//      tiles, as in layer 2;
//   2. after a barrier the partial sums go to LDS (over the a2 tile, 12 bytes per (row, dz,
//      voxel)) and y(v) = sum over (dz, dy) of P[(dz, dy)] at row (y + dy, z + dz): nine LDS
//      reads per output, summed in a fixed order.
// Per 512 outputs: 120 MFMAs and 34.6 KB of LDS for the tile (four blocks per CU).
constexpr int kL3Rows = kHY * kHZ;                 // 60 input rows
constexpr int kL3RowsPerWave = kL3Rows / (kBlk / 64);  // 15
static_assert(kL3Rows % (kBlk / 64) == 0, "every wavefront takes the same number of rows");
static_assert(kL3Rows * 3 * kBX * 3 * 4 <= 2 * kHalf * 16, "the partial sums fit over the a2 tile");

__global__ void __launch_bounds__(kBlk) k_net_l3m(const uint16_t* __restrict__ a2, const u32x4* __restrict__ w3l,
                                                  const int N, const int mode, const double* __restrict__ ssum,
                                                  float* __restrict__ y) {
  __shared__ u32x4 tile[2 * kHalf];
  int x0, y0, z0;
  brick_of(N, x0, y0, z0);
  fill_halo_tile(reinterpret_cast<const u32x4*>(a2), N, x0, y0, z0, tile);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 15, g = lane >> 4;
  const u32x4 wA1 = w3l[lane], wA2 = w3l[64 + lane];
  __syncthreads();
  // stage 1: rows j = wave + 4 k of the 60; slot g >> 1 of the first B is dx = -1 or 0, both
  // slots of the second dx = +1 (its second slot meets zero weights)
  const u32x4* t1 = tile + (g & 1) * kHalf + col + (g >> 1);
  const u32x4* t2 = tile + (g & 1) * kHalf + col + 2;
  floatx4 p[kL3RowsPerWave];
#pragma unroll
  for (int k = 0; k < kL3RowsPerWave; ++k) {
    const int j = wave + 4 * k;  // row hy + kHY hz of the halo'd brick
    p[k] = mfma32(wA1, t1[j * kHX], floatx4{0.0f, 0.0f, 0.0f, 0.0f});
    p[k] = mfma32(wA2, t2[j * kHX], p[k]);
  }
  __builtin_amdgcn_iglp_opt(0);
  __syncthreads();
  // lane (col, g < 3) holds P[(dz = g - 1, dy = -1, 0, 1)] of voxel col of its rows
  float* pl = reinterpret_cast<float*>(tile);  // [row][dz][x][dy]
  if (g < 3) {
#pragma unroll
    for (int k = 0; k < kL3RowsPerWave; ++k) {
      const int j = wave + 4 * k;
      float* d = pl + ((j * 3 + g) * kBX + col) * 3;
      d[0] = p[k][0];
      d[1] = p[k][1];
      d[2] = p[k][2];
    }
  }
  __syncthreads();
  // stage 2: thread (x, ty, tz pair) sums its two outputs over (dz, dy)
  const int x = threadIdx.x & 15, ty = (threadIdx.x >> 4) & 7, tz0 = 2 * (threadIdx.x >> 7);
  float acc[2];
#pragma unroll
  for (int o = 0; o < 2; ++o) {
    const int tz = tz0 + o;
    float s = 0.0f;
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const int j = (tz + dz) * kHY + (ty + dy);  // input row (ty + 1 + dy - 1, tz + 1 + dz - 1)
        s += pl[((j * 3 + dz) * kBX + x) * 3 + dy];
      }
    acc[o] = s;
  }
  float sc = 1.0f;
  if (mode != 0) {
    const double nn = static_cast<double>(N) * N * N;
    sc = static_cast<float>(sqrt(*ssum / nn));
  }
#pragma unroll
  for (int o = 0; o < 2; ++o) {
    float* dst = y + vox(x0 + x, y0 + ty, z0 + tz0 + o, N);
    if (mode == 0) *dst = acc[o];
    else *dst += sc * acc[o];
  }
}

// planes per segment of k_net_l3s: segments of at least 16 planes, enough blocks to fill the device
inline int l3s_segments(int N) {
  const int cols = (N / kSX) * (N / kSY);
  int nseg = 1;
  while (cols * nseg < 4096 && N / (2 * nseg) >= 16) nseg *= 2;
  return nseg;
}

// 16 BF16 channels of one voxel (32 bytes) to FP32
__device__ __forceinline__ void load16(const uint16_t* p, float* f) {
  const uint4* q = reinterpret_cast<const uint4*>(p);
  const uint4 a = q[0], b = q[1];
  const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    f[2 * c] = __uint_as_float(w[c] << 16);
    f[2 * c + 1] = __uint_as_float(w[c] & 0xFFFF0000u);
  }
}

// ---------------------------------------------------------------------------- backward
// g2[v][c] = bf16(1[a2[v][c] > 0] sum_t W3[c][t] gy[v - off(t)])
__global__ void __launch_bounds__(kBlk) k_net_l3_bwd(const float* __restrict__ gy, const uint16_t* __restrict__ a2,
                                                     const float* __restrict__ w3q, const int N,
                                                     uint16_t* __restrict__ g2) {
  __shared__ float w[kTaps * kNC];
  for (int e = threadIdx.x; e < kTaps * kNC; e += kBlk) w[e] = w3q[e];
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y, k = blockIdx.z;
  if (i >= N) return;
  float g[kNC];
#pragma unroll
  for (int c = 0; c < kNC; ++c) g[c] = 0.0f;
#pragma unroll
  for (int t = 0; t < kTaps; ++t) {
    const float gv = gy[nbr(i, j, k, t, -1, N)];
#pragma unroll
    for (int c = 0; c < kNC; ++c) g[c] = fmaf(w[t * kNC + c], gv, g[c]);
  }
  const size_t v = vox(i, j, k, N);
  float a[kNC];
  load16(a2 + v * kNC, a);
  uint32_t p[kNC / 2];
#pragma unroll
  for (int c = 0; c < kNC / 2; ++c) {
    const float lo = a[2 * c] > 0.0f ? g[2 * c] : 0.0f;
    const float hi = a[2 * c + 1] > 0.0f ? g[2 * c + 1] : 0.0f;
    p[c] = static_cast<uint32_t>(f2bf(lo)) | (static_cast<uint32_t>(f2bf(hi)) << 16);
  }
  uint4* dst = reinterpret_cast<uint4*>(g2 + v * kNC);
  dst[0] = make_uint4(p[0], p[1], p[2], p[3]);
  dst[1] = make_uint4(p[4], p[5], p[6], p[7]);
}

// gin[v] = sum_t sum_c W1[c][t] g1[v - off(t)][c]
__global__ void __launch_bounds__(kBlk) k_net_gin(const uint16_t* __restrict__ g1, const float* __restrict__ w1q,
                                                  const int N, float* __restrict__ gin) {
  __shared__ float w[kTaps * kNC];
  for (int e = threadIdx.x; e < kTaps * kNC; e += kBlk) w[e] = w1q[e];
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y, k = blockIdx.z;
  if (i >= N) return;
  float acc = 0.0f;
#pragma unroll 3
  for (int t = 0; t < kTaps; ++t) {
    float g[kNC];
    load16(g1 + nbr(i, j, k, t, -1, N) * kNC, g);
#pragma unroll
    for (int c = 0; c < kNC; ++c) acc = fmaf(w[t * kNC + c], g[c], acc);
  }
  gin[vox(i, j, k, N)] = acc;
}

// Weight gradients of layers 1 and 3 (16 values per tap), one partial per
// (block, tap):  layer 3: sum_v gy[v] a2[v + off(t)][c];
//                layer 1: sum_v g1[v][c] x_in[v + off(t)].
constexpr int kWgChunk = 4096;  // voxels per block

template <int LAYER>
__global__ void __launch_bounds__(kBlk) k_net_wgrad13(const float* __restrict__ gy, const uint16_t* __restrict__ a2,
                                                      const uint16_t* __restrict__ g1,
                                                      const uint16_t* __restrict__ xin, const int N,
                                                      float* __restrict__ part) {
  __shared__ float red[kBlk][kNC + 1];
  const int t = blockIdx.y;
  const size_t nv = static_cast<size_t>(N) * N * N;
  const size_t v0 = static_cast<size_t>(blockIdx.x) * kWgChunk;
  float acc[kNC];
#pragma unroll
  for (int c = 0; c < kNC; ++c) acc[c] = 0.0f;
  for (size_t v = v0 + threadIdx.x; v < v0 + kWgChunk && v < nv; v += kBlk) {
    const int i = static_cast<int>(v % N);
    const int j = static_cast<int>((v / N) % N);
    const int k = static_cast<int>(v / (static_cast<size_t>(N) * N));
    const size_t u = nbr(i, j, k, t, 1, N);
    float f[kNC];
    if (LAYER == 3) {
      const float g = gy[v];
      load16(a2 + u * kNC, f);
#pragma unroll
      for (int c = 0; c < kNC; ++c) acc[c] = fmaf(g, f[c], acc[c]);
    } else {
      const float x = bf2f(xin[u]);
      load16(g1 + v * kNC, f);
#pragma unroll
      for (int c = 0; c < kNC; ++c) acc[c] = fmaf(f[c], x, acc[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < kNC; ++c) red[threadIdx.x][c] = acc[c];
  __syncthreads();
  for (int s = kBlk / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
#pragma unroll
      for (int c = 0; c < kNC; ++c) red[threadIdx.x][c] += red[threadIdx.x + s][c];
    __syncthreads();
  }
  if (threadIdx.x < kNC) part[(static_cast<size_t>(blockIdx.x) * kTaps + t) * kNC + threadIdx.x] = red[0][threadIdx.x];
}

// Layer-2 weight gradient on the matrix cores (v_mfma_f32_16x16x32_bf16): for each tap,
// D[o][i] += sum over 32-voxel groups of G^T (16 o x 32 voxels) X_t (32 voxels x 16 i),
// G = g2, X_t = a1 shifted by the tap.  Each wavefront sums kW2Vox voxels and writes one
// partial of 27 x 256 values.
constexpr int kW2Vox = 2048;

__global__ void __launch_bounds__(kBlk) k_net_wgrad2(const uint16_t* __restrict__ g2, const uint16_t* __restrict__ a1,
                                                     const int N, float* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int wv = blockIdx.x * (kBlk / 64) + (threadIdx.x >> 6);
  const size_t nv = static_cast<size_t>(N) * N * N;
  const size_t v0 = static_cast<size_t>(wv) * kW2Vox;
  const int col = lane & 15, g = lane >> 4;
  floatx4 acc[kTaps];
#pragma unroll
  for (int t = 0; t < kTaps; ++t) acc[t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  for (size_t g0 = v0; g0 < v0 + kW2Vox && g0 < nv; g0 += 32) {
    // this lane's voxels g0 + 8 g + e, e = 0 .. 7 (N^3 is a multiple of 32)
    int vi[8], vj[8], vk[8];
    uint32_t av[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const size_t v = g0 + 8 * g + e;
      vi[e] = static_cast<int>(v % N);
      vj[e] = static_cast<int>((v / N) % N);
      vk[e] = static_cast<int>(v / (static_cast<size_t>(N) * N));
      av[e] = g2[v * kNC + col];  // A[m = o = col][k = voxel]
    }
    const u32x4 a{av[0] | (av[1] << 16), av[2] | (av[3] << 16), av[4] | (av[5] << 16), av[6] | (av[7] << 16)};
#pragma unroll
    for (int t = 0; t < kTaps; ++t) {
      // B[k = voxel][n = i = col] = a1[voxel + off(t)][col]
      uint32_t bv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) bv[e] = a1[nbr(vi[e], vj[e], vk[e], t, 1, N) * kNC + col];
      const u32x4 b{bv[0] | (bv[1] << 16), bv[2] | (bv[3] << 16), bv[4] | (bv[5] << 16), bv[6] | (bv[7] << 16)};
      acc[t] = mfma32(a, b, acc[t]);
    }
  }
  // D[o = 4 g + r][i = col]
  float* dst = part + static_cast<size_t>(wv) * kTaps * kNC * kNC;
#pragma unroll
  for (int t = 0; t < kTaps; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) dst[(t * kNC + 4 * g + r) * kNC + col] = acc[t][r];
}

// gw[base + (o * nin + i) * 27 + t] += sum_p part[p][t][o][i]   (fixed order)
__global__ void __launch_bounds__(kBlk) k_net_reduce(const float* __restrict__ part, const int np, const int nout,
                                                     const int nin, float* __restrict__ gw, const int base) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = kTaps * nout * nin;
  if (e >= per) return;
  const int t = e / (nout * nin), oi = e % (nout * nin);
  double s = 0.0;
  for (int p = 0; p < np; ++p) s += part[static_cast<size_t>(p) * per + e];
  gw[base + oi * kTaps + t] += static_cast<float>(s);
}

// ---------------------------------------------------------------------------- weights
// Flat master layout: W1[co][t] (432), W2[co][ci][t] (6912), W3[ci][t] (432).
// Kernel layouts: w1q[t][co], w3q[t][ci] (BF16-rounded values as FP32),
// w2f[t][co][ci] (forward A operand), w2b[t'][ci][co] with t' the mirrored tap
// (backward-data A operand).
__global__ void __launch_bounds__(kBlk) k_net_pack(const float* __restrict__ w, float* __restrict__ w1q,
                                                   uint16_t* __restrict__ w2f, uint16_t* __restrict__ w2b,
                                                   float* __restrict__ w3q) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < 432) {
    const int co = e / kTaps, t = e % kTaps;
    w1q[t * kNC + co] = bf2f(f2bf(w[e]));
  } else if (e < 432 + 6912) {
    const int f = e - 432;
    const int co = f / (kNC * kTaps), ci = (f / kTaps) % kNC, t = f % kTaps;
    const uint16_t h = f2bf(w[e]);
    w2f[(t * kNC + co) * kNC + ci] = h;
    w2b[((kTaps - 1 - t) * kNC + ci) * kNC + co] = h;
  } else if (e < 7776) {
    const int f = e - 432 - 6912;
    const int ci = f / kTaps, t = f % kTaps;
    w3q[t * kNC + ci] = bf2f(f2bf(w[e]));
  }
}

// Lane-ordered copies of the MFMA A operands, one 16-byte entry per (operand, lane), so a lane
// loads each operand with one load at a fixed offset:
//   w2fl / w2bl  entry (p * 3 + dy) * 64 + l: w2f / w2b[t][l & 15][8h .. 8h + 7] for the tap t of
//                (dz, dx) pair p, slot (l >> 4) >> 1, and dy (h = (l >> 4) & 1), zero for the empty
//                slot of the last pair (see load_l2_weights);
//   w1l          entry l: W1 taps of (dz, dy) rows 2g and 2g + 1 (dx = -1, 0, 1, then a zero, each)
//                for output channel l & 15, g = l >> 4; entry 64 + l: row 8 in group 0, else zero.
__global__ void __launch_bounds__(kBlk) k_net_pack_lanes(const uint16_t* __restrict__ w2f,
                                                         const uint16_t* __restrict__ w2b,
                                                         const float* __restrict__ w1q,
                                                         const float* __restrict__ w3q, u32x4* __restrict__ w2fl,
                                                         u32x4* __restrict__ w2bl, u32x4* __restrict__ w1l,
                                                         u32x4* __restrict__ w3l) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < kPairs * 3 * 64) {
    const int l = e % 64, pd = e / 64, p = pd / 3, dy = pd % 3;
    const int col = l & 15, g = l >> 4, h = g & 1, c = 2 * p + (g >> 1);
    u32x4 f{0u, 0u, 0u, 0u}, bk{0u, 0u, 0u, 0u};
    if (c < 9) {
      const int t = (c / 3) * 9 + dy * 3 + (c % 3);
      f = *reinterpret_cast<const u32x4*>(w2f + (t * kNC + col) * kNC + 8 * h);
      bk = *reinterpret_cast<const u32x4*>(w2b + (t * kNC + col) * kNC + 8 * h);
    }
    w2fl[e] = f;
    w2bl[e] = bk;
  } else if (e < kPairs * 3 * 64 + 128) {
    const int f = e - kPairs * 3 * 64;
    const int l = f % 64, col = l & 15, g = l >> 4;
    auto wt = [&](int t) { return w1q[t * kNC + col]; };
    if (f < 64) {
      const int ra = 2 * g, rb = 2 * g + 1;
      w1l[f] = u32x4{pack2(wt(3 * ra), wt(3 * ra + 1)), pack2(wt(3 * ra + 2), 0.0f), pack2(wt(3 * rb), wt(3 * rb + 1)),
                     pack2(wt(3 * rb + 2), 0.0f)};
    } else {
      w1l[f] = g == 0 ? u32x4{pack2(wt(24), wt(25)), pack2(wt(26), 0.0f), 0u, 0u} : u32x4{0u, 0u, 0u, 0u};
    }
  } else if (e < kPairs * 3 * 64 + 256) {
    // layer 3 (k_net_l3s, k_net_l3m): entry l: row m = l & 15 = 4 (dz + 1) + (dy + 1), k group g = l >> 4,
    // channels 8 (g & 1) .. +7 of dx = (g >> 1) - 1; entry 64 + l: dx = +1 in slot 0, zero in slot 1
    const int f = e - kPairs * 3 * 64 - 128;
    const int l = f % 64, m = l & 15, g = l >> 4, h = g & 1, slot = g >> 1;
    const int dz = m / 4 - 1, dy = m % 4 - 1;
    const int dx = f < 64 ? slot - 1 : (slot == 0 ? 1 : 2);
    float w[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (dz <= 1 && dy <= 1 && dx <= 1) {
      const int t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
#pragma unroll
      for (int j = 0; j < 8; ++j) w[j] = w3q[t * kNC + 8 * h + j];
    }
    w3l[f] = u32x4{pack2(w[0], w[1]), pack2(w[2], w[3]), pack2(w[4], w[5]), pack2(w[6], w[7])};
  }
}

// Adam (Kingma and Ba 2015) on the FP32 master weights.
__global__ void __launch_bounds__(kBlk) k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v2,
                                               const float* __restrict__ g, const int n, const float lr,
                                               const float b1, const float b2, const float eps, const float c1,
                                               const float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gg = g[e];
  const float mm = b1 * m[e] + (1.0f - b1) * gg;
  const float vv = b2 * v2[e] + (1.0f - b2) * gg * gg;
  m[e] = mm;
  v2[e] = vv;
  w[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// et = s y with s = sqrt(ssum / N^3)
__global__ void __launch_bounds__(kBlk) k_scale_s(const float* __restrict__ y, const double* __restrict__ ssum,
                                                  const int64_t n, float* __restrict__ et) {
  const float s = static_cast<float>(sqrt(*ssum / static_cast<double>(n)));
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    et[i] = s * y[i];
}

// gy = coef d with coef = -2 s scale / (e^T r): the gradient of
// ||e - s y||_A^2 / ||e||_A^2 with respect to y, given d = r - A s y and A e = r.
__global__ void __launch_bounds__(kBlk) k_loss_gy(const float* __restrict__ d, const double* __restrict__ ssum,
                                                  const double* __restrict__ er, const double scale, const int64_t n,
                                                  float* __restrict__ gy) {
  const double s = sqrt(*ssum / static_cast<double>(n));
  const float coef = static_cast<float>(-2.0 * s * scale / *er);
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    gy[i] = coef * d[i];
}

inline dim3 vgrid(int N) { return dim3((N + kBlk - 1) / kBlk, N, N); }
inline dim3 in_grid(int N) { return dim3((N / 4 + kInThreads - 1) / kInThreads, N, N); }

ClassTab64 ctab(const double* t, int q) {
  ClassTab64 c{};
  for (int i = 0; i < q * q * q; ++i) c.v[i] = t[i];
  return c;
}

}  // namespace

int64_t net_cache_bytes(int N) {
  const int64_t nv = static_cast<int64_t>(N) * N * N;
  const int64_t a = (nv * 2 + 255) / 256 * 256;
  return a + 2 * nv * kNC * 2;
}

int64_t net_partial_floats(int N) {
  const int64_t nv = static_cast<int64_t>(N) * N * N;
  const int64_t waves = (nv + kW2Vox - 1) / kW2Vox;
  const int64_t w2 = ((waves + 3) / 4) * 4 * kTaps * kNC * kNC;
  const int64_t w13 = ((nv + kWgChunk - 1) / kWgChunk) * kTaps * kNC;
  return w2 > w13 ? w2 : w13;
}

hipError_t launch_net_pack(const float* w, NetDev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_net_pack, dim3((7776 + kBlk - 1) / kBlk), dim3(kBlk), 0, s, w, d.w1q, d.w2f, d.w2b, d.w3q);
  hipLaunchKernelGGL(k_net_pack_lanes, dim3((kPairs * 3 * 64 + 256 + kBlk - 1) / kBlk), dim3(kBlk), 0, s, d.w2f,
                     d.w2b, d.w1q, d.w3q, reinterpret_cast<u32x4*>(d.w2fl), reinterpret_cast<u32x4*>(d.w2bl),
                     reinterpret_cast<u32x4*>(d.w1l), reinterpret_cast<u32x4*>(d.w3l));
  return hipGetLastError();
}

hipError_t launch_net_input(const float* r, const double* dinv, int q, const double* ssum, double* part,
                            int64_t part_cap, int N, void* cache, hipStream_t s) {
  uint16_t* xin = static_cast<uint16_t*>(cache);
  // rows are read four values at a time
  if (N % 4 != 0 || reinterpret_cast<uintptr_t>(r) % 16 != 0 || reinterpret_cast<uintptr_t>(cache) % 16 != 0)
    return hipErrorInvalidValue;
  if (dinv) {
    const ClassTab64 c = ctab(dinv, q);
    const int sq_threads = std::min(kBlk, std::max(64, (N / 4 + 63) / 64 * 64));
    hipLaunchKernelGGL(k_net_sqsum, dim3(1, N, N), dim3(sq_threads), 0, s, r, c, q, N, part);
    const hipError_t e = launch_sum_partials(part, static_cast<int64_t>(N) * N, part_cap, const_cast<double*>(ssum), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_net_in, in_grid(N), dim3(kInThreads), 0, s, r, c, q, 1, ssum, N, xin);
  } else {
    const ClassTab64 c{};
    hipLaunchKernelGGL(k_net_in, in_grid(N), dim3(kInThreads), 0, s, r, c, q, 0, ssum, N, xin);
  }
  return hipGetLastError();
}

hipError_t launch_net_forward(const NetDev& d, int N, void* cache, int mode, const double* ssum, float* y,
                              hipStream_t s, bool keep_a1) {
  if (N < 16 || (N & (N - 1)) != 0) return hipErrorInvalidValue;
  const int64_t nv = static_cast<int64_t>(N) * N * N;
  uint16_t* xin = static_cast<uint16_t*>(cache);
  uint16_t* a1 = reinterpret_cast<uint16_t*>(static_cast<char*>(cache) + (nv * 2 + 255) / 256 * 256);
  uint16_t* a2 = a1 + nv * kNC;
  const int nb = (N / kBX) * (N / kBY) * (N / kBZ);
  if (keep_a1)
    hipLaunchKernelGGL(k_net_l12<true>, dim3(nb), dim3(kBlk), 0, s, xin, reinterpret_cast<const u32x4*>(d.w1l),
                       reinterpret_cast<const u32x4*>(d.w2fl), N, a1, a2);
  else
    hipLaunchKernelGGL(k_net_l12<false>, dim3(nb), dim3(kBlk), 0, s, xin, reinterpret_cast<const u32x4*>(d.w1l),
                       reinterpret_cast<const u32x4*>(d.w2fl), N, nullptr, a2);
  if (N >= 128) {  // streamed along z (at 512^3 voxels 1.33 against 1.71 ms)
    const int nseg = l3s_segments(N);
    hipLaunchKernelGGL(k_net_l3s, dim3((N / kSX) * (N / kSY) * nseg), dim3(kBlk), 0, s, a2,
                       reinterpret_cast<const u32x4*>(d.w3l), N, nseg, mode, ssum, y);
  } else {  // one pass over bricks (on 16^3 to 64^3 voxels 35-49 against 52-65 us a correction)
    hipLaunchKernelGGL(k_net_l3m, dim3(nb), dim3(kBlk), 0, s, a2, reinterpret_cast<const u32x4*>(d.w3l), N, mode,
                       ssum, y);
  }
  return hipGetLastError();
}

hipError_t launch_net_backward(const NetDev& d, int N, const void* cache, const float* gy, void* g1g2, float* part,
                               float* gw, float* gin, hipStream_t s) {
  if (N < 16 || (N & (N - 1)) != 0) return hipErrorInvalidValue;
  const int64_t nv = static_cast<int64_t>(N) * N * N;
  const uint16_t* xin = static_cast<const uint16_t*>(cache);
  const uint16_t* a1 = reinterpret_cast<const uint16_t*>(static_cast<const char*>(cache) + (nv * 2 + 255) / 256 * 256);
  const uint16_t* a2 = a1 + nv * kNC;
  uint16_t* g2 = static_cast<uint16_t*>(g1g2);
  uint16_t* g1 = g2 + nv * kNC;
  hipLaunchKernelGGL(k_net_l3_bwd, vgrid(N), dim3(kBlk), 0, s, gy, a2, d.w3q, N, g2);
  const int nb = (N / kBX) * (N / kBY) * (N / kBZ);
  hipLaunchKernelGGL(k_net_l2bwd, dim3(nb), dim3(kBlk), 0, s, g2, reinterpret_cast<const u32x4*>(d.w2bl), a1, N,
                     g1);
  // layer 3 weights
  const int nch = static_cast<int>((nv + kWgChunk - 1) / kWgChunk);
  hipLaunchKernelGGL(k_net_wgrad13<3>, dim3(nch, kTaps), dim3(kBlk), 0, s, gy, a2, nullptr, nullptr, N, part);
  hipLaunchKernelGGL(k_net_reduce, dim3((kTaps * kNC + kBlk - 1) / kBlk), dim3(kBlk), 0, s, part, nch, 1, kNC, gw,
                     432 + 6912);
  // layer 2 weights (MFMA)
  const int nw = static_cast<int>((nv + kW2Vox - 1) / kW2Vox);
  const int nwb = (nw + 3) / 4;
  hipLaunchKernelGGL(k_net_wgrad2, dim3(nwb), dim3(kBlk), 0, s, g2, a1, N, part);
  hipLaunchKernelGGL(k_net_reduce, dim3((kTaps * kNC * kNC + kBlk - 1) / kBlk), dim3(kBlk), 0, s, part, nwb * 4,
                     kNC, kNC, gw, 432);
  // layer 1 weights
  hipLaunchKernelGGL(k_net_wgrad13<1>, dim3(nch, kTaps), dim3(kBlk), 0, s, nullptr, nullptr, g1, xin, N, part);
  hipLaunchKernelGGL(k_net_reduce, dim3((kTaps * kNC + kBlk - 1) / kBlk), dim3(kBlk), 0, s, part, nch, kNC, 1, gw,
                     0);
  if (gin) hipLaunchKernelGGL(k_net_gin, vgrid(N), dim3(kBlk), 0, s, g1, d.w1q, N, gin);
  return hipGetLastError();
}

hipError_t launch_net_scale(const float* y, const double* ssum, int64_t n, float* et, hipStream_t s) {
  const int g = static_cast<int>(std::min<int64_t>((n + kBlk * 4 - 1) / (kBlk * 4), 65535));
  hipLaunchKernelGGL(k_scale_s, dim3(g), dim3(kBlk), 0, s, y, ssum, n, et);
  return hipGetLastError();
}

hipError_t launch_net_loss_gy(const float* d, const double* ssum, const double* er, double scale, int64_t n, float* gy,
                              hipStream_t s) {
  const int g = static_cast<int>(std::min<int64_t>((n + kBlk * 4 - 1) / (kBlk * 4), 65535));
  hipLaunchKernelGGL(k_loss_gy, dim3(g), dim3(kBlk), 0, s, d, ssum, er, scale, n, gy);
  return hipGetLastError();
}

hipError_t launch_adam(NetDev& d, const float* gw, float lr, int64_t step, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.0f - powf(b1, static_cast<float>(step));
  const float c2 = 1.0f - powf(b2, static_cast<float>(step));
  hipLaunchKernelGGL(k_adam, dim3((7776 + kBlk - 1) / kBlk), dim3(kBlk), 0, s, d.w, d.m, d.v, gw, 7776, lr, b1, b2,
                     eps, c1, c2);
  return launch_net_pack(d.w, d, s);
}

}  // namespace gmg
