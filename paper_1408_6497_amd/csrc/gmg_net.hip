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
//   k_net_l12  one 16x8x4 brick per block: bf16(x) with a two-voxel halo in LDS;
//              layer 1 on the matrix cores over the brick plus a one-voxel halo
//              (27 taps padded to K = 32); a1 stays in LDS; layer 2 (6912 of the
//              7776 multiply-adds per voxel) on v_mfma_f32_16x16x16_bf16 with the
//              16x16 weight block of a tap as A (registers, all 27 taps) and 16
//              input channels x 16 voxels along x as B (from the LDS tile),
//              accumulating 16 output channels x 16 voxels over the 27 taps; a2
//              to HBM (32 B per voxel), a1 only when training keeps it.
//   k_net_l3t  layer 3 over the same bricks from an LDS tile of a2, two voxels
//              per thread, with the output update u += s y fused.
// The backward-data pass of layer 2 is k_net_l2 with the flipped, transposed
// weights and the ReLU mask of the forward pass.
#include <algorithm>

#include "gmg_kernels.h"

namespace gmg {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

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
__device__ __forceinline__ uint32_t pack2(float a, float b) {
  const bf16x2 v = {static_cast<__bf16>(a), static_cast<__bf16>(b)};
  return __builtin_bit_cast(uint32_t, v);
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
// x_in = bf16(D^-1 r / s) with s = sqrt(ssum / N^3) (or x_in = bf16(x) when dinv is null)
__global__ void __launch_bounds__(kBlk) k_net_in(const float* __restrict__ r, const ClassTab64 dinv, const int q,
                                                 const int use_dinv, const double* __restrict__ ssum, const int N,
                                                 uint16_t* __restrict__ xin) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y, k = blockIdx.z;
  if (i >= N) return;
  const size_t v = vox(i, j, k, N);
  float x = r[v];
  if (use_dinv) {
    const double nn = static_cast<double>(N) * N * N;
    const float s = static_cast<float>(sqrt(*ssum / nn));
    const float d = static_cast<float>(dinv.v[(i % q) + q * ((j % q) + q * (k % q))]);
    x = (s > 0.0f) ? (d * x) / s : 0.0f;
  }
  xin[v] = f2bf(x);
}

// sum over voxels of (D^-1 r)^2, one partial per (j, k) row
__global__ void __launch_bounds__(kBlk) k_net_sqsum(const float* __restrict__ r, const ClassTab64 dinv, const int q,
                                                    const int N, double* part) {
  __shared__ double red[kBlk / 64];
  const int j = blockIdx.y, k = blockIdx.z;
  double s = 0.0;
  const float* row = r + (static_cast<size_t>(k) * N + j) * N;
  const int base = q * ((j % q) + q * (k % q));
  for (int i = threadIdx.x; i < N; i += kBlk) {
    const float d = static_cast<float>(dinv.v[base + i % q]);
    const double t = static_cast<double>(d * row[i]);
    s = fma(t, t, s);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlk / 64; ++w) t += red[w];
    part[static_cast<size_t>(k) * N + j] = t;
  }
}

// ---------------------------------------------------------------------------- layer 2 (16 -> 16, MFMA)
constexpr int kBX = 16, kBY = 8, kBZ = 4;
constexpr int kHX = kBX + 2, kHY = kBY + 2, kHZ = kBZ + 2;

// out[v][m] = sum_t sum_k wA[t][m][k] in[v + off(t)][k];  forward: bf16(relu(.)),
// backward-data (MASK): bf16(. * 1[mask[v][m] > 0]).  N >= 16.
template <bool MASK>
__global__ void __launch_bounds__(kBlk) k_net_l2(const uint16_t* __restrict__ in, const uint16_t* __restrict__ wA,
                                                 const uint16_t* __restrict__ mask, const int N,
                                                 uint16_t* __restrict__ out) {
  __shared__ uint2 tile[kHZ * kHY * kHX * 4];  // 4 x (4 bf16) per voxel
  const int nbx = N / kBX, nby = N / kBY;
  const int b = blockIdx.x;
  const int x0 = (b % nbx) * kBX;
  const int y0 = ((b / nbx) % nby) * kBY;
  const int z0 = (b / (nbx * nby)) * kBZ;
  const int m = N - 1;
  const uint2* in2 = reinterpret_cast<const uint2*>(in);
  for (int e = threadIdx.x; e < kHZ * kHY * kHX * 4; e += kBlk) {
    const int c = e & 3;
    const int vx = e >> 2;
    const int hx = vx % kHX, hy = (vx / kHX) % kHY, hz = vx / (kHX * kHY);
    const size_t g = vox((x0 - 1 + hx) & m, (y0 - 1 + hy) & m, (z0 - 1 + hz) & m, N);
    tile[e] = in2[g * 4 + c];
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 15;   // A row (output channel) / B column (voxel)
  const int kb = lane >> 4;    // k block: input channels 4 kb .. 4 kb + 3
  bf16x4 wa[kTaps];
  const uint2* wA2 = reinterpret_cast<const uint2*>(wA);
#pragma unroll
  for (int t = 0; t < kTaps; ++t) {
    const uint2 u = wA2[(t * kNC + col) * 4 + kb];
    wa[t] = *reinterpret_cast<const bf16x4*>(&u);
  }
  __syncthreads();
  for (int tt = wave; tt < kBY * kBZ; tt += kBlk / 64) {
    const int ty = tt % kBY, tz = tt / kBY;
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < kTaps; ++t) {
      const int dx = (t % 3) - 1, dy = ((t / 3) % 3) - 1, dz = (t / 9) - 1;
      const int hidx = ((tz + 1 + dz) * kHY + (ty + 1 + dy)) * kHX + (col + 1 + dx);
      const uint2 u = tile[hidx * 4 + kb];
      const bf16x4 bv = *reinterpret_cast<const bf16x4*>(&u);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[t], bv, acc, 0, 0, 0);
    }
    // lane holds output channels 4 kb .. 4 kb + 3 of voxel (x0 + col, y0 + ty, z0 + tz)
    const size_t v = vox(x0 + col, y0 + ty, z0 + tz, N);
    float o[4];
    if (MASK) {
      const uint2 mk = reinterpret_cast<const uint2*>(mask)[v * 4 + kb];
      const uint16_t mv[4] = {static_cast<uint16_t>(mk.x & 0xFFFF), static_cast<uint16_t>(mk.x >> 16),
                              static_cast<uint16_t>(mk.y & 0xFFFF), static_cast<uint16_t>(mk.y >> 16)};
#pragma unroll
      for (int r = 0; r < 4; ++r) o[r] = bf2f(mv[r]) > 0.0f ? acc[r] : 0.0f;
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) o[r] = fmaxf(acc[r], 0.0f);
    }
    uint2 pk;
    pk.x = static_cast<uint32_t>(f2bf(o[0])) | (static_cast<uint32_t>(f2bf(o[1])) << 16);
    pk.y = static_cast<uint32_t>(f2bf(o[2])) | (static_cast<uint32_t>(f2bf(o[3])) << 16);
    reinterpret_cast<uint2*>(out)[v * 4 + kb] = pk;
  }
}

// ---------------------------------------------------------------------------- fused layers 1 + 2
// One block per 16x8x4 output brick.  bf16(x) of the brick plus a two-voxel halo
// goes to LDS; layer 1 runs on the matrix cores over the brick plus a one-voxel
// halo (27 taps as K = 32: two v_mfma_f32_16x16x16_bf16 per 16 voxels, W1 as A,
// the taps of 16 voxels as B), ReLU and BF16 rounding, into an LDS tile of the
// same layout layer 2 reads; layer 2 then runs as in k_net_l2.  a1 never goes to
// HBM unless the caller keeps it (training: the backward pass reads it).
constexpr int kXX = kBX + 4, kXY = kBY + 4, kXZ = kBZ + 4;  // input tile with a two-voxel halo
constexpr int kHalo = kHX * kHY * kHZ;                      // 1080 voxels of layer 1 output

template <bool KEEP_A1>
__global__ void __launch_bounds__(kBlk) k_net_l12(const uint16_t* __restrict__ xin, const float* __restrict__ w1q,
                                                  const uint16_t* __restrict__ wA, const int N,
                                                  uint16_t* __restrict__ a1_out, uint16_t* __restrict__ a2_out) {
  __shared__ uint16_t xt[kXZ * kXY * kXX];
  __shared__ uint2 tile[kHalo * 4];
  const int nbx = N / kBX, nby = N / kBY;
  const int b = blockIdx.x;
  const int x0 = (b % nbx) * kBX;
  const int y0 = ((b / nbx) % nby) * kBY;
  const int z0 = (b / (nbx * nby)) * kBZ;
  const int m = N - 1;
  for (int e = threadIdx.x; e < kXZ * kXY * kXX; e += kBlk) {
    const int hx = e % kXX, hy = (e / kXX) % kXY, hz = e / (kXX * kXY);
    xt[e] = xin[vox((x0 - 2 + hx) & m, (y0 - 2 + hy) & m, (z0 - 2 + hz) & m, N)];
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 15;
  const int kb = lane >> 4;
  // W1 as the A operand: row = output channel col, k = taps 16 j + 4 kb + r
  bf16x4 w1a[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    short h[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int t = 16 * j + 4 * kb + r;
      h[r] = t < kTaps ? static_cast<short>(f2bf(w1q[t * kNC + col])) : static_cast<short>(0);
    }
    w1a[j] = bf16x4{h[0], h[1], h[2], h[3]};
  }
  bf16x4 wa[kTaps];
  const uint2* wA2 = reinterpret_cast<const uint2*>(wA);
#pragma unroll
  for (int t = 0; t < kTaps; ++t) {
    const uint2 u = wA2[(t * kNC + col) * 4 + kb];
    wa[t] = *reinterpret_cast<const bf16x4*>(&u);
  }
  __syncthreads();
  // per-lane tap offsets in the input tile: taps 16 j + 4 kb + r (taps >= 27 read zero)
  int toff[8];
  bool tuse[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int t = 16 * (i >> 2) + 4 * kb + (i & 3);
    tuse[i] = t < kTaps;
    const int dx = (t % 3) - 1, dy = ((t / 3) % 3) - 1, dz = (t / 9) - 1;
    toff[i] = tuse[i] ? (dz * kXY + dy) * kXX + dx : 0;
  }
  // layer 1 over the 1080 voxels of the brick plus a one-voxel halo, 16 at a time
  for (int g = wave; g < (kHalo + 15) / 16; g += kBlk / 64) {
    const int e = 16 * g + col;
    const bool live = e < kHalo;
    const int ec = live ? e : kHalo - 1;
    const int hz = ec / (kHX * kHY);
    const int rem = ec - hz * (kHX * kHY);
    const int hy = rem / kHX;
    const int hx = rem - hy * kHX;
    const int base = ((hz + 1) * kXY + (hy + 1)) * kXX + (hx + 1);
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      short h[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) h[r] = tuse[4 * j + r] ? static_cast<short>(xt[base + toff[4 * j + r]]) : short(0);
      const bf16x4 bv{h[0], h[1], h[2], h[3]};
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1a[j], bv, acc, 0, 0, 0);
    }
    // lane holds output channels 4 kb .. 4 kb + 3 of voxel e
    uint2 pk;
    pk.x = pack2(fmaxf(acc[0], 0.0f), fmaxf(acc[1], 0.0f));
    pk.y = pack2(fmaxf(acc[2], 0.0f), fmaxf(acc[3], 0.0f));
    if (live) {
      tile[e * 4 + kb] = pk;
      if (KEEP_A1 && hx >= 1 && hx <= kBX && hy >= 1 && hy <= kBY && hz >= 1 && hz <= kBZ)
        reinterpret_cast<uint2*>(a1_out)[vox(x0 + hx - 1, y0 + hy - 1, z0 + hz - 1, N) * 4 + kb] = pk;
    }
  }
  __syncthreads();
  // layer 2: wave tz owns the 8 output rows of plane tz (16 channels x 16 voxels
  // each).  Every a1 row loaded from LDS feeds the up to three output rows it is
  // a y-neighbour of, so the tile is read 90 times per wave instead of 216.
  static_assert(kBlk / 64 == kBZ, "one wave per plane of the brick");
  const int tz = wave;
  floatx4 acc[kBY];
#pragma unroll
  for (int ty = 0; ty < kBY; ++ty) acc[ty] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx)
#pragma unroll
      for (int r = 0; r < kHY; ++r) {
        const uint2 u = tile[(((tz + 1 + dz) * kHY + r) * kHX + (col + 1 + dx)) * 4 + kb];
        const bf16x4 bv = *reinterpret_cast<const bf16x4*>(&u);
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
          const int ty = r - 1 - dy;
          if (ty < 0 || ty >= kBY) continue;
          const int t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
          acc[ty] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[t], bv, acc[ty], 0, 0, 0);
        }
      }
#pragma unroll
  for (int ty = 0; ty < kBY; ++ty) {
    const size_t v = vox(x0 + col, y0 + ty, z0 + tz, N);
    uint2 pk;
    pk.x = pack2(fmaxf(acc[ty][0], 0.0f), fmaxf(acc[ty][1], 0.0f));
    pk.y = pack2(fmaxf(acc[ty][2], 0.0f), fmaxf(acc[ty][3], 0.0f));
    reinterpret_cast<uint2*>(a2_out)[v * 4 + kb] = pk;
  }
}

// ---------------------------------------------------------------------------- layer 3, LDS-tiled
// y = W3 * a2 over one 16x8x4 brick: a2 of the brick plus a one-voxel halo in LDS,
// each thread two neighbouring voxels along x (the 4 x-columns they need are read
// once for both).  Channel pairs go through v_dot2c_f32_bf16 (two BF16 products
// added to the FP32 accumulator) straight from the packed activations; the sum
// runs over taps t = 0..26, then channel pairs.  Tile rows are padded by 16 bytes
// so the 128-bit reads of neighbouring rows fall on different LDS banks.
constexpr int kRowU2 = kHX * 4 + 2;  // uint2 per padded tile row

__device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float c) {
  return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, a), __builtin_bit_cast(bf16x2, b), c, false);
}

__global__ void __launch_bounds__(kBlk) k_net_l3t(const uint16_t* __restrict__ a2, const float* __restrict__ w3q,
                                                  const int N, const int mode, const double* __restrict__ ssum,
                                                  float* __restrict__ y) {
  __shared__ __align__(16) uint2 tile[kHZ * kHY * kRowU2];
  __shared__ uint32_t w[kTaps * kNC / 2];  // [t][channel pair], BF16 pairs
  const int nbx = N / kBX, nby = N / kBY;
  const int b = blockIdx.x;
  const int x0 = (b % nbx) * kBX;
  const int y0 = ((b / nbx) % nby) * kBY;
  const int z0 = (b / (nbx * nby)) * kBZ;
  const int m = N - 1;
  const uint2* in2 = reinterpret_cast<const uint2*>(a2);
  for (int e = threadIdx.x; e < kHalo * 4; e += kBlk) {
    const int c = e & 3;
    const int vx = e >> 2;
    const int hx = vx % kHX, hy = (vx / kHX) % kHY, hz = vx / (kHX * kHY);
    tile[(hz * kHY + hy) * kRowU2 + hx * 4 + c] =
        in2[vox((x0 - 1 + hx) & m, (y0 - 1 + hy) & m, (z0 - 1 + hz) & m, N) * 4 + c];
  }
  for (int e = threadIdx.x; e < kTaps * kNC / 2; e += kBlk)
    w[e] = static_cast<uint32_t>(f2bf(w3q[2 * e])) | (static_cast<uint32_t>(f2bf(w3q[2 * e + 1])) << 16);
  __syncthreads();
  const int xp = threadIdx.x & 7;          // voxel pair along x
  const int ty = (threadIdx.x >> 3) & 7;
  const int tz = threadIdx.x >> 6;
  const int hx0 = 2 * xp;                   // halo column of x - 1 for the first voxel
  float acc0 = 0.0f, acc1 = 0.0f;
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int rowb = ((tz + 1 + dz) * kHY + (ty + 1 + dy)) * kRowU2;
      uint32_t a[4][kNC / 2];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint4* q = reinterpret_cast<const uint4*>(tile + rowb + (hx0 + k) * 4);
        const uint4 u0 = q[0], u1 = q[1];
        a[k][0] = u0.x;
        a[k][1] = u0.y;
        a[k][2] = u0.z;
        a[k][3] = u0.w;
        a[k][4] = u1.x;
        a[k][5] = u1.y;
        a[k][6] = u1.z;
        a[k][7] = u1.w;
      }
      const int tb = (dz + 1) * 9 + (dy + 1) * 3;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const uint32_t* wt = w + (tb + dx) * (kNC / 2);
#pragma unroll
        for (int c = 0; c < kNC / 2; ++c) {
          acc0 = dot2(a[dx][c], wt[c], acc0);
          acc1 = dot2(a[dx + 1][c], wt[c], acc1);
        }
      }
    }
  const size_t v = vox(x0 + 2 * xp, y0 + ty, z0 + tz, N);
  if (mode == 0) {
    y[v] = acc0;
    y[v + 1] = acc1;
  } else {
    const double nn = static_cast<double>(N) * N * N;
    const float sc = static_cast<float>(sqrt(*ssum / nn));
    y[v] += sc * acc0;
    y[v + 1] += sc * acc1;
  }
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

// Layer-2 weight gradient on the matrix cores: for each tap,
// D[o][i] += sum over 16-voxel groups of G^T (16 o x 16 voxels) X_t (16 voxels x 16 i),
// G = g2, X_t = a1 shifted by the tap.  Each wavefront sums kW2Vox voxels and
// writes one partial of 27 x 256 values.
constexpr int kW2Vox = 2048;

__global__ void __launch_bounds__(kBlk) k_net_wgrad2(const uint16_t* __restrict__ g2, const uint16_t* __restrict__ a1,
                                                     const int N, float* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int wv = blockIdx.x * (kBlk / 64) + (threadIdx.x >> 6);
  const size_t nv = static_cast<size_t>(N) * N * N;
  const size_t v0 = static_cast<size_t>(wv) * kW2Vox;
  const int col = lane & 15, kb = lane >> 4;
  floatx4 acc[kTaps];
#pragma unroll
  for (int t = 0; t < kTaps; ++t) acc[t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  for (size_t g = v0; g < v0 + kW2Vox && g < nv; g += 16) {
    // group of 16 consecutive voxels along x (N is a multiple of 16)
    const int i0 = static_cast<int>(g % N);
    const int j = static_cast<int>((g / N) % N);
    const int k = static_cast<int>(g / (static_cast<size_t>(N) * N));
    // A[m = o = col][kk = voxel 4 kb + r] = g2[g + 4 kb + r][col]
    short av[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) av[r] = static_cast<short>(g2[(g + 4 * kb + r) * kNC + col]);
    const bf16x4 a = {av[0], av[1], av[2], av[3]};
#pragma unroll
    for (int t = 0; t < kTaps; ++t) {
      // B[kk = voxel 4 kb + r][n = i = col] = a1[(voxel + off(t))][col]
      short bv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) bv[r] = static_cast<short>(a1[nbr(i0 + 4 * kb + r, j, k, t, 1, N) * kNC + col]);
      const bf16x4 b = {bv[0], bv[1], bv[2], bv[3]};
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
    }
  }
  // D[o = 4 kb + r][i = col]
  float* dst = part + static_cast<size_t>(wv) * kTaps * kNC * kNC;
#pragma unroll
  for (int t = 0; t < kTaps; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) dst[(t * kNC + 4 * kb + r) * kNC + col] = acc[t][r];
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
  return hipGetLastError();
}

hipError_t launch_net_input(const float* r, const double* dinv, int q, const double* ssum, double* part,
                            int64_t part_cap, int N, void* cache, hipStream_t s) {
  uint16_t* xin = static_cast<uint16_t*>(cache);
  if (dinv) {
    const ClassTab64 c = ctab(dinv, q);
    hipLaunchKernelGGL(k_net_sqsum, dim3(1, N, N), dim3(kBlk), 0, s, r, c, q, N, part);
    const hipError_t e = launch_sum_partials(part, static_cast<int64_t>(N) * N, part_cap, const_cast<double*>(ssum), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_net_in, vgrid(N), dim3(kBlk), 0, s, r, c, q, 1, ssum, N, xin);
  } else {
    const ClassTab64 c{};
    hipLaunchKernelGGL(k_net_in, vgrid(N), dim3(kBlk), 0, s, r, c, q, 0, ssum, N, xin);
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
    hipLaunchKernelGGL(k_net_l12<true>, dim3(nb), dim3(kBlk), 0, s, xin, d.w1q, d.w2f, N, a1, a2);
  else
    hipLaunchKernelGGL(k_net_l12<false>, dim3(nb), dim3(kBlk), 0, s, xin, d.w1q, d.w2f, N, nullptr, a2);
  hipLaunchKernelGGL(k_net_l3t, dim3(nb), dim3(kBlk), 0, s, a2, d.w3q, N, mode, ssum, y);
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
  hipLaunchKernelGGL(k_net_l2<true>, dim3(nb), dim3(kBlk), 0, s, g2, d.w2b, a1, N, g1);
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
