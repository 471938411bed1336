// Reductions, vector updates, node-class scalings and the coarsest solve.
//
// Reductions accumulate in FP64 whatever the vector type: 64-lane wavefront
// shuffles, then LDS across the block, then a second single-block pass over the
// per-block partials in a fixed order (deterministic results).
#include <mutex>

#include "gmg_kernels.h"

namespace gmg {
namespace {

constexpr int kBlock = 256;

inline int grid_for(int64_t n, int per_thread = 4) {
  int64_t g = (n + static_cast<int64_t>(kBlock) * per_thread - 1) / (static_cast<int64_t>(kBlock) * per_thread);
  if (g < 1) g = 1;
  if (g > 65535) g = 65535;
  return static_cast<int>(g);
}

// ---------------------------------------------------------------- class tables
struct ClassTab {
  double v[kMaxQ * kMaxQ * kMaxQ];
};

// Node-class kernels run on a (ceil(N/256), N, N) grid: x along the row, y and z
// from the block index, so the class (i mod q, j mod q, k mod q) needs no 64-bit
// division.
struct Ijk {
  int i, j, k;
  size_t idx;
};

__device__ __forceinline__ bool ijk_of(int N, Ijk* p) {
  p->i = blockIdx.x * blockDim.x + threadIdx.x;
  p->j = blockIdx.y;
  p->k = blockIdx.z;
  p->idx = (static_cast<size_t>(p->k) * N + p->j) * N + p->i;
  return p->i < N;
}

__device__ __forceinline__ int cls(const Ijk& p, int q) { return (p.i % q) + q * ((p.j % q) + q * (p.k % q)); }

inline dim3 class_grid(int N) { return dim3((N + kBlock - 1) / kBlock, N, N); }

template <typename T>
__global__ void __launch_bounds__(kBlock) k_class_scale(const ClassTab tab, const int q, const int N, const double c,
                                                         const T* in, T* out) {
  Ijk p;
  if (!ijk_of(N, &p)) return;
  const double v = in ? static_cast<double>(in[p.idx]) : 1.0;
  out[p.idx] = static_cast<T>(c * tab.v[cls(p, q)] * v);
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < kBlock / 64; ++w) s += red[w];
  }
  return s;  // valid in thread 0
}

// Each thread visits i, i + S, i + 2 S, ... (S = threads in the grid) in that order and
// sums in that order; the loads of four visits are issued before their products, so
// more bytes are in flight per thread than in the one-visit loop (same sums, bit for bit).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dot(const int64_t n, const T* __restrict__ x, const T* __restrict__ y,
                                                 double* part) {
  double s = 0.0;
  const int64_t S = static_cast<int64_t>(gridDim.x) * blockDim.x;
  int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  for (; i + 3 * S < n; i += 4 * S) {
    T xv[4], yv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      xv[k] = x[i + k * S];
      yv[k] = y ? y[i + k * S] : T(1);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) s = fma(static_cast<double>(xv[k]), static_cast<double>(yv[k]), s);
  }
  for (; i < n; i += S) s = fma(static_cast<double>(x[i]), static_cast<double>(y ? y[i] : T(1)), s);
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// sum_i tab[class(i)] x_i: each block sums a plane-row strip, blocks write
// partials in a fixed order (grid (1, N, N) -> N^2 partials, folded by k_finish_many).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_class_dot(const ClassTab tab, const int q, const int N,
                                                       const T* __restrict__ x, double* part) {
  const int j = blockIdx.y, k = blockIdx.z;
  const T* row = x + (static_cast<size_t>(k) * N + j) * N;
  double s = 0.0;
  const int base = q * ((j % q) + q * (k % q));
  for (int i = threadIdx.x; i < N; i += kBlock) s = fma(tab.v[base + i % q], static_cast<double>(row[i]), s);
  s = block_sum(s);
  if (threadIdx.x == 0) part[static_cast<size_t>(k) * N + j] = s;
}

__global__ void __launch_bounds__(kBlock) k_finish(const double* part, const int nparts, double* dst) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kBlock) s += part[i];
  s = block_sum(s);
  if (threadIdx.x == 0) *dst = s;
}

// Three block sums at once (valid in thread 0): one LDS round, no reuse hazard.
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c) {
  __shared__ double red[3][kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
    c += __shfl_down(c, off, 64);
  }
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wid] = a;
    red[1][wid] = b;
    red[2][wid] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = b = c = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) {
      a += red[0][w];
      b += red[1][w];
      c += red[2][w];
    }
  }
}

// Fused reductions of the Krylov loop.  Each block writes its partials to
// (x.x, y.y) in one pass, visiting as k_dot does
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sq2(const int64_t n, const T* __restrict__ x, const T* __restrict__ y,
                                                 double* part) {
  double a = 0.0, b = 0.0, c = 0.0;
  const int64_t S = static_cast<int64_t>(gridDim.x) * blockDim.x;
  int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  for (; i + 3 * S < n; i += 4 * S) {
    T xv[4], yv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      xv[k] = x[i + k * S];
      yv[k] = y[i + k * S];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a = fma(static_cast<double>(xv[k]), static_cast<double>(xv[k]), a);
      b = fma(static_cast<double>(yv[k]), static_cast<double>(yv[k]), b);
    }
  }
  for (; i < n; i += S) {
    a = fma(static_cast<double>(x[i]), static_cast<double>(x[i]), a);
    b = fma(static_cast<double>(y[i]), static_cast<double>(y[i]), b);
  }
  block_sum3(a, b, c);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a;
    part[gridDim.x + blockIdx.x] = b;
  }
}

// part[k * nblocks + block] (k = 0, 1, 2); k_finish_multi folds them in a fixed order.
// (x.y, x.z)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dot2(const int64_t n, const T* __restrict__ x, const T* __restrict__ y,
                                                 const T* __restrict__ z, double* part) {
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double xv = static_cast<double>(x[i]);
    a = fma(xv, static_cast<double>(y[i]), a);
    b = fma(xv, static_cast<double>(z[i]), b);
  }
  block_sum3(a, b, c);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a;
    part[gridDim.x + blockIdx.x] = b;
  }
}

// (x.y, x.z, sum y): the FCG step's two products and the sum of w = A p, whose
// mean predicts the mean of the updated residual
__global__ void __launch_bounds__(kBlock) k_dot2_sumy(const int64_t n, const double* __restrict__ x,
                                                      const double* __restrict__ y, const double* __restrict__ z,
                                                      double* part) {
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double xv = x[i];
    const double yv = y[i];
    a = fma(xv, yv, a);
    b = fma(xv, z[i], b);
    c += yv;
  }
  block_sum3(a, b, c);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a;
    part[gridDim.x + blockIdx.x] = b;
    part[2 * gridDim.x + blockIdx.x] = c;
  }
}

// FCG update with the projection and the cast to the cycle's precision in the same
// pass: alpha = sc[inum] / sc[iden], u += alpha p, r <- r - alpha w - m, r32 = float(r),
// partial sum(r) and r.r of the stored r.  m = (sc[irs] - alpha sc[iws]) scale is the
// mean of r - alpha w predicted from sum(r) (sc[irs]) and sum(w) (sc[iws]), so the
// stored residual stays mean-free to rounding without a pass of its own; its exact
// sum goes back to sc[irs] for the norm and the next prediction.
__global__ void __launch_bounds__(kBlock) k_axpy2_cast(const int64_t n, const double* sc, const int inum,
                                                       const int iden, const int irs, const int iws,
                                                       const double scale, double* u, const double* __restrict__ p,
                                                       double* r, const double* __restrict__ w,
                                                       float* __restrict__ r32, double* part) {
  const double al = sc[inum] / sc[iden];
  const double m = (sc[irs] - al * sc[iws]) * scale;
  double a = 0.0, b = 0.0, c = 0.0;
  // visits in k_dot's order, the loads of four visits issued together
  const int64_t S = static_cast<int64_t>(gridDim.x) * blockDim.x;
  int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  for (; i + 3 * S < n; i += 4 * S) {
    double uv[4], pv[4], rv[4], wv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      uv[k] = u[i + k * S];
      pv[k] = p[i + k * S];
      rv[k] = r[i + k * S];
      wv[k] = w[i + k * S];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      u[i + k * S] = fma(al, pv[k], uv[k]);
      const double v = fma(-al, wv[k], rv[k]) - m;
      r[i + k * S] = v;
      r32[i + k * S] = static_cast<float>(v);
      a += v;
      b = fma(v, v, b);
    }
  }
  for (; i < n; i += S) {
    u[i] = fma(al, p[i], u[i]);
    const double v = fma(-al, w[i], r[i]) - m;
    r[i] = v;
    r32[i] = static_cast<float>(v);
    a += v;
    b = fma(v, v, b);
  }
  block_sum3(a, b, c);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a;
    part[gridDim.x + blockIdx.x] = b;
  }
}

// u += alpha p, r -= alpha w (alpha = sc[inum] / sc[iden]); partial sum(r) and r.r of the new r
template <typename T>
__global__ void __launch_bounds__(kBlock) k_axpy2_sums(const int64_t n, const double* sc, const int inum,
                                                       const int iden, T* u, const T* __restrict__ p, T* r,
                                                       const T* __restrict__ w, double* part) {
  const T al = static_cast<T>(sc[inum] / sc[iden]);
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    u[i] = fma(al, p[i], u[i]);
    const T rn = fma(-al, w[i], r[i]);
    r[i] = rn;
    const double rd = static_cast<double>(rn);
    a += rd;
    b = fma(rd, rd, b);
  }
  block_sum3(a, b, c);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a;
    part[gridDim.x + blockIdx.x] = b;
  }
}

// (sum z, z.y, sum y)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sums3(const int64_t n, const T* __restrict__ z, const T* __restrict__ y,
                                                  double* part) {
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double zv = static_cast<double>(z[i]);
    const double yv = static_cast<double>(y[i]);
    a += zv;
    b = fma(zv, yv, b);
    c += yv;
  }
  block_sum3(a, b, c);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a;
    part[gridDim.x + blockIdx.x] = b;
    part[2 * gridDim.x + blockIdx.x] = c;
  }
}

// (sum z, z.y, sum y) with z the FP32 output of a cycle and y an FP64 Krylov vector
__global__ void __launch_bounds__(kBlock) k_sums3_mixed(const int64_t n, const float* __restrict__ z,
                                                        const double* __restrict__ y, double* part) {
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double zv = static_cast<double>(z[i]);
    const double yv = y[i];
    a += zv;
    b = fma(zv, yv, b);
    c += yv;
  }
  block_sum3(a, b, c);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a;
    part[gridDim.x + blockIdx.x] = b;
    part[2 * gridDim.x + blockIdx.x] = c;
  }
}

// (sum z, z.w, sum w, z.r) with z the FP32 output of a cycle, w and r FP64 Krylov vectors
__global__ void __launch_bounds__(kBlock) k_sums4_mixed(const int64_t n, const float* __restrict__ z,
                                                        const double* __restrict__ w, const double* __restrict__ r,
                                                        double* part) {
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double zv = static_cast<double>(z[i]);
    const double wv = w[i];
    a += zv;
    b = fma(zv, wv, b);
    c += wv;
    d = fma(zv, r[i], d);
  }
  double e = 0.0, f = 0.0;
  block_sum3(a, b, c);
  __syncthreads();  // block_sum3's LDS is reused below
  block_sum3(d, e, f);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a;
    part[gridDim.x + blockIdx.x] = b;
    part[2 * gridDim.x + blockIdx.x] = c;
    part[3 * gridDim.x + blockIdx.x] = d;
  }
}

// sc[d_k] = sum of the k-th run of nparts partials (one block per k, k < 4)
__global__ void __launch_bounds__(kBlock) k_finish_multi(const double* part, const int nparts, double* sc,
                                                         const int d0, const int d1, const int d2, const int d3 = 0) {
  const int k = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kBlock) s += part[static_cast<size_t>(k) * nparts + i];
  double u = 0.0, v = 0.0;
  block_sum3(s, u, v);
  if (threadIdx.x == 0) sc[k == 0 ? d0 : (k == 1 ? d1 : (k == 2 ? d2 : d3))] = s;
}

// sc[dst] = sc[a] - sc[b] sc[c] scale   (one thread)
__global__ void k_combine(double* sc, const int dst, const int a, const int b, const int c, const double scale) {
  if (threadIdx.x == 0 && blockIdx.x == 0) sc[dst] = sc[a] - sc[b] * sc[c] * scale;
}

// p = (z - sc[imean] scale) + beta p,  beta = sgn sc[inum] / sc[iden]
template <typename T>
__global__ void __launch_bounds__(kBlock) k_xpby_shift(const int64_t n, const double* sc, const int inum,
                                                       const int iden, const double sgn, const int imean,
                                                       const double scale, const T* __restrict__ z, T* p) {
  const T be = static_cast<T>(sgn * sc[inum] / sc[iden]);
  const T m = static_cast<T>(sc[imean] * scale);
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = fma(be, p[i], z[i] - m);
}

// p = (z - sc[imean] scale) + beta p with z the FP32 output of a cycle, p FP64
__global__ void __launch_bounds__(kBlock) k_xpby_shift_mixed(const int64_t n, const double* sc, const int inum,
                                                             const int iden, const double sgn, const int imean,
                                                             const double scale, const float* __restrict__ z,
                                                             double* p) {
  const double be = sgn * sc[inum] / sc[iden];
  const double m = sc[imean] * scale;
  const int64_t S = static_cast<int64_t>(gridDim.x) * blockDim.x;
  int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  for (; i + 3 * S < n; i += 4 * S) {
    double pv[4];
    float zv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      pv[k] = p[i + k * S];
      zv[k] = z[i + k * S];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) p[i + k * S] = fma(be, pv[k], static_cast<double>(zv[k]) - m);
  }
  for (; i < n; i += S) p[i] = fma(be, p[i], static_cast<double>(z[i]) - m);
}

// r -= sc[i0] scale, r32 = float(r), and the partial sums of squares and of the
// values of the new r (the squares in the same grid and order as a separate
// dot(r, r) after the shift)
__global__ void __launch_bounds__(kBlock) k_shift_cast_sq(const int64_t n, const double* sc, const int i0,
                                                          const double scale, const double* src, double* r,
                                                          float* __restrict__ r32, double* part) {
  const double m = sc[i0] * scale;
  double s = 0.0, t = 0.0, u = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double v = src[i] - m;
    r[i] = v;
    r32[i] = static_cast<float>(v);
    s = fma(v, v, s);
    t += v;
  }
  block_sum3(s, t, u);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s;
    part[gridDim.x + blockIdx.x] = t;
  }
}

// u = 0 and the partial sums of b and of b^2 (the start of a solve from a zero guess)
__global__ void __launch_bounds__(kBlock) k_zero_sums(const int64_t n, const double* __restrict__ b,
                                                      double* __restrict__ u, double* part) {
  double s = 0.0, q = 0.0, t = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double v = b[i];
    u[i] = 0.0;
    s += v;
    q = fma(v, v, q);
  }
  block_sum3(s, q, t);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s;
    part[gridDim.x + blockIdx.x] = q;
  }
}

// p = double(z) - sc[i0] scale: the first direction from an FP32 cycle output
__global__ void __launch_bounds__(kBlock) k_shift_f2d(const int64_t n, const double* sc, const int i0,
                                                      const double scale, const float* __restrict__ z,
                                                      double* __restrict__ p) {
  const double m = sc[i0] * scale;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = static_cast<double>(z[i]) - m;
}

// Sum of a long run of partials in two fixed-order passes: `blocks` blocks fold
// contiguous chunks into part2, one block folds those.
__global__ void __launch_bounds__(kBlock) k_fold(const double* part, const int64_t nparts, const int64_t chunk,
                                                 double* part2) {
  const int64_t b0 = blockIdx.x * chunk;
  const int64_t b1 = b0 + chunk < nparts ? b0 + chunk : nparts;
  double s = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += kBlock) s += part[i];
  s = block_sum(s);
  if (threadIdx.x == 0) part2[blockIdx.x] = s;
}

inline int red_grid(int64_t n) {
  int g = grid_for(n, 8);
  return g > kRedBlocks ? kRedBlocks : g;
}

// ---------------------------------------------------------------- vector updates
template <typename T>
__global__ void __launch_bounds__(kBlock) k_axpy2(const int64_t n, const double* sc, const int inum, const int iden,
                                                   T* u, const T* __restrict__ p, T* r, const T* __restrict__ w) {
  const T a = static_cast<T>(sc[inum] / sc[iden]);
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    u[i] = fma(a, p[i], u[i]);
    r[i] = fma(-a, w[i], r[i]);
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_xpby(const int64_t n, const double* sc, const int inum, const int iden,
                                                  const double sgn, const T* __restrict__ z, T* p) {
  const T b = static_cast<T>(sgn * sc[inum] / sc[iden]);
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = fma(b, p[i], z[i]);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_shift(const int64_t n, const double* sc, const int i0, const double scale,
                                                   T* v) {
  const T m = static_cast<T>(sc[i0] * scale);
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    v[i] -= m;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_axpy(const int64_t n, const double a, const T* __restrict__ x,
                                                  T* __restrict__ y) {
  const T aa = static_cast<T>(a);
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    y[i] = fma(aa, x[i], y[i]);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_class_axpy(const ClassTab tab, const int q, const int N, const double c,
                                                        T* v) {
  Ijk p;
  if (!ijk_of(N, &p)) return;
  v[p.idx] = static_cast<T>(static_cast<double>(v[p.idx]) + c * tab.v[cls(p, q)]);
}

// SplitMix64 (Steele, Lea, Flood 2014): output i of the stream with key k.
__global__ void __launch_bounds__(kBlock) k_splitmix_start(const uint64_t key, const int64_t n, double* out) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    uint64_t z = key + static_cast<uint64_t>(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    out[i] = 2.0 * static_cast<double>(z >> 11) * 0x1.0p-53 - 1.0;
  }
}

__global__ void __launch_bounds__(kBlock) k_cast_d2f(const int64_t n, const double* __restrict__ in,
                                                      float* __restrict__ out) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[i] = static_cast<float>(in[i]);
}

__global__ void __launch_bounds__(kBlock) k_cast_f2d(const int64_t n, const float* __restrict__ in,
                                                      double* __restrict__ out) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[i] = static_cast<double>(in[i]);
}

__global__ void __launch_bounds__(kBlock) k_add_f2d(const int64_t n, const float* __restrict__ c,
                                                     double* __restrict__ u) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    u[i] += static_cast<double>(c[i]);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill_zero(const int64_t n, T* v) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    v[i] = T(0);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_copy(const int64_t n, const T* __restrict__ in, T* __restrict__ out) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[i] = in[i];
}

// ---------------------------------------------------------------- coarsest solve
// x = Ainv (b - mean(b)) with Ainv symmetric (row i read contiguously): each
// block has 4 wavefronts, one row each; every block recomputes the mean of b
// (n0 <= 4096 values, held in dynamic LDS of 8 n0 bytes) so no second launch is needed.
constexpr int kCoarseMax = 4096;
constexpr int kCoarseRows = 4;

template <typename T>
__global__ void __launch_bounds__(64 * kCoarseRows) k_coarse(const int n0, const double* __restrict__ ainv,
                                                              const T* __restrict__ b, T* __restrict__ x) {
  extern __shared__ double bs[];
  __shared__ double red[kCoarseRows];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double s = 0.0;
  for (int i = threadIdx.x; i < n0; i += 64 * kCoarseRows) {
    const double v = static_cast<double>(b[i]);
    bs[i] = v;
    s += v;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) red[w] = s;
  __syncthreads();
  double tot = 0.0;
  for (int k = 0; k < kCoarseRows; ++k) tot += red[k];
  const double m = tot / n0;
  const int row = blockIdx.x * kCoarseRows + w;
  if (row >= n0) return;
  const double* arow = ainv + static_cast<size_t>(row) * n0;
  double acc = 0.0;
  for (int j = lane; j < n0; j += 64) acc = fma(arow[j], bs[j] - m, acc);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) x[row] = static_cast<T>(acc);
}

}  // namespace

hipError_t launch_class_scale(bool fp32, int q, int N, const double* tab, double c, const void* in, void* out,
                              hipStream_t s) {
  ClassTab ct{};
  for (int i = 0; i < q * q * q; ++i) ct.v[i] = tab[i];
  if (fp32)
    hipLaunchKernelGGL(k_class_scale<float>, class_grid(N), dim3(kBlock), 0, s, ct, q, N, c,
                       static_cast<const float*>(in), static_cast<float*>(out));
  else
    hipLaunchKernelGGL(k_class_scale<double>, class_grid(N), dim3(kBlock), 0, s, ct, q, N, c,
                       static_cast<const double*>(in), static_cast<double*>(out));
  return hipGetLastError();
}

hipError_t launch_dot(bool fp32, int64_t n, const void* x, const void* y, double* part, double* dst, hipStream_t s) {
  const int g = red_grid(n);
  if (fp32)
    hipLaunchKernelGGL(k_dot<float>, dim3(g), dim3(kBlock), 0, s, n, static_cast<const float*>(x),
                       static_cast<const float*>(y), part);
  else
    hipLaunchKernelGGL(k_dot<double>, dim3(g), dim3(kBlock), 0, s, n, static_cast<const double*>(x),
                       static_cast<const double*>(y), part);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kBlock), 0, s, part, g, dst);
  return hipGetLastError();
}

}  // namespace gmg

// ------------------------------------------------------------ the no-allocation dot
// Partials of the first pass of gmg_dot_noalloc live in this file-scope device array
// (one copy per device, held until the process ends), not in memory the library
// allocates.  In host code `scratch` names a host-side stand-in, so its device address
// is taken once per device with hipGetSymbolAddress at setup and only that address is
// passed to kernels.
static __device__ __align__(256) double scratch[gmg::kNoallocPartials];

namespace gmg {
namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (p == nullptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

hipError_t launch_dot_noalloc(int device, bool fp32, int64_t n, const void* x, const void* y, double* dst,
                              hipStream_t s) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  void* p = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    p = g_scratch_ptr[device];
  }
  if (p == nullptr) return hipErrorNotInitialized;
  // the first pass writes one partial per block, every block, so nothing in the scratch
  // needs clearing between calls; its block count must fit the scratch
  if (red_grid(n) > kNoallocPartials) return hipErrorInvalidValue;
  return launch_dot(fp32, n, x, y, static_cast<double*>(p), dst, s);
}

hipError_t launch_sq2(bool fp32, int64_t n, const void* x, const void* y, double* part, double* sc, int dx, int dy,
                      hipStream_t s) {
  const int g = red_grid(n);
  if (fp32)
    hipLaunchKernelGGL(k_sq2<float>, dim3(g), dim3(kBlock), 0, s, n, static_cast<const float*>(x),
                       static_cast<const float*>(y), part);
  else
    hipLaunchKernelGGL(k_sq2<double>, dim3(g), dim3(kBlock), 0, s, n, static_cast<const double*>(x),
                       static_cast<const double*>(y), part);
  hipLaunchKernelGGL(k_finish_multi, dim3(2), dim3(kBlock), 0, s, part, g, sc, dx, dy, 0);
  return hipGetLastError();
}

hipError_t launch_dot2(bool fp32, int64_t n, const void* x, const void* y, const void* z, double* part, double* sc,
                       int dxy, int dxz, hipStream_t s) {
  const int g = red_grid(n);
  if (fp32)
    hipLaunchKernelGGL(k_dot2<float>, dim3(g), dim3(kBlock), 0, s, n, static_cast<const float*>(x),
                       static_cast<const float*>(y), static_cast<const float*>(z), part);
  else
    hipLaunchKernelGGL(k_dot2<double>, dim3(g), dim3(kBlock), 0, s, n, static_cast<const double*>(x),
                       static_cast<const double*>(y), static_cast<const double*>(z), part);
  hipLaunchKernelGGL(k_finish_multi, dim3(2), dim3(kBlock), 0, s, part, g, sc, dxy, dxz, 0);
  return hipGetLastError();
}

hipError_t launch_axpy2_sums(bool fp32, int64_t n, double* sc, int inum, int iden, void* u, const void* p, void* r,
                             const void* w, double* part, int dsum, int dsq, hipStream_t s) {
  const int g = red_grid(n);
  if (fp32)
    hipLaunchKernelGGL(k_axpy2_sums<float>, dim3(g), dim3(kBlock), 0, s, n, sc, inum, iden, static_cast<float*>(u),
                       static_cast<const float*>(p), static_cast<float*>(r), static_cast<const float*>(w), part);
  else
    hipLaunchKernelGGL(k_axpy2_sums<double>, dim3(g), dim3(kBlock), 0, s, n, sc, inum, iden,
                       static_cast<double*>(u), static_cast<const double*>(p), static_cast<double*>(r),
                       static_cast<const double*>(w), part);
  hipLaunchKernelGGL(k_finish_multi, dim3(2), dim3(kBlock), 0, s, part, g, sc, dsum, dsq, 0);
  return hipGetLastError();
}

hipError_t launch_sums3(bool fp32, int64_t n, const void* z, const void* y, double* part, double* sc, int dz,
                        int dzy, int dy, hipStream_t s) {
  const int g = red_grid(n);
  if (fp32)
    hipLaunchKernelGGL(k_sums3<float>, dim3(g), dim3(kBlock), 0, s, n, static_cast<const float*>(z),
                       static_cast<const float*>(y), part);
  else
    hipLaunchKernelGGL(k_sums3<double>, dim3(g), dim3(kBlock), 0, s, n, static_cast<const double*>(z),
                       static_cast<const double*>(y), part);
  hipLaunchKernelGGL(k_finish_multi, dim3(3), dim3(kBlock), 0, s, part, g, sc, dz, dzy, dy);
  return hipGetLastError();
}

hipError_t launch_sums3_mixed(int64_t n, const float* z, const double* y, double* part, double* sc, int dz, int dzy,
                              int dy, hipStream_t s) {
  const int g = red_grid(n);
  hipLaunchKernelGGL(k_sums3_mixed, dim3(g), dim3(kBlock), 0, s, n, z, y, part);
  hipLaunchKernelGGL(k_finish_multi, dim3(3), dim3(kBlock), 0, s, part, g, sc, dz, dzy, dy);
  return hipGetLastError();
}

hipError_t launch_sums4_mixed(int64_t n, const float* z, const double* w, const double* r, double* part, double* sc,
                              int dz, int dzw, int dw, int dzr, hipStream_t s) {
  const int g = red_grid(n);
  hipLaunchKernelGGL(k_sums4_mixed, dim3(g), dim3(kBlock), 0, s, n, z, w, r, part);
  hipLaunchKernelGGL(k_finish_multi, dim3(4), dim3(kBlock), 0, s, part, g, sc, dz, dzw, dw, dzr);
  return hipGetLastError();
}

hipError_t launch_xpby_shift_mixed(int64_t n, const double* sc, int inum, int iden, double sgn, int imean,
                                   double scale, const float* z, double* p, hipStream_t s) {
  hipLaunchKernelGGL(k_xpby_shift_mixed, dim3(grid_for(n)), dim3(kBlock), 0, s, n, sc, inum, iden, sgn, imean, scale,
                     z, p);
  return hipGetLastError();
}

hipError_t launch_shift_cast_sq(int64_t n, double* sc, int i, double scale, const double* src, double* r, float* r32,
                                double* part, int dsq, int dsum, hipStream_t s) {
  const int g = red_grid(n);
  hipLaunchKernelGGL(k_shift_cast_sq, dim3(g), dim3(kBlock), 0, s, n, sc, i, scale, src, r, r32, part);
  hipLaunchKernelGGL(k_finish_multi, dim3(2), dim3(kBlock), 0, s, part, g, sc, dsq, dsum, 0);
  return hipGetLastError();
}

hipError_t launch_zero_sums(int64_t n, const double* b, double* u, double* part, double* sc, int dsum, int dsq,
                            hipStream_t s) {
  const int g = red_grid(n);
  hipLaunchKernelGGL(k_zero_sums, dim3(g), dim3(kBlock), 0, s, n, b, u, part);
  hipLaunchKernelGGL(k_finish_multi, dim3(2), dim3(kBlock), 0, s, part, g, sc, dsum, dsq, 0);
  return hipGetLastError();
}

hipError_t launch_dot2_sumy(int64_t n, const double* x, const double* y, const double* z, double* part, double* sc,
                            int dxy, int dxz, int dy, hipStream_t s) {
  const int g = red_grid(n);
  hipLaunchKernelGGL(k_dot2_sumy, dim3(g), dim3(kBlock), 0, s, n, x, y, z, part);
  hipLaunchKernelGGL(k_finish_multi, dim3(3), dim3(kBlock), 0, s, part, g, sc, dxy, dxz, dy);
  return hipGetLastError();
}

hipError_t launch_axpy2_cast(int64_t n, double* sc, int inum, int iden, int irs, int iws, double scale, double* u,
                             const double* p, double* r, const double* w, float* r32, double* part, int dsq,
                             hipStream_t s) {
  const int g = red_grid(n);
  hipLaunchKernelGGL(k_axpy2_cast, dim3(g), dim3(kBlock), 0, s, n, sc, inum, iden, irs, iws, scale, u, p, r, w, r32,
                     part);
  hipLaunchKernelGGL(k_finish_multi, dim3(2), dim3(kBlock), 0, s, part, g, sc, irs, dsq, 0);
  return hipGetLastError();
}

hipError_t launch_shift_f2d(int64_t n, const double* sc, int i, double scale, const float* z, double* p,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_shift_f2d, dim3(grid_for(n)), dim3(kBlock), 0, s, n, sc, i, scale, z, p);
  return hipGetLastError();
}

hipError_t launch_combine(double* sc, int dst, int a, int b, int c, double scale, hipStream_t s) {
  hipLaunchKernelGGL(k_combine, dim3(1), dim3(64), 0, s, sc, dst, a, b, c, scale);
  return hipGetLastError();
}

hipError_t launch_xpby_shift(bool fp32, int64_t n, const double* sc, int inum, int iden, double sgn, int imean,
                             double scale, const void* z, void* p, hipStream_t s) {
  const int g = grid_for(n);
  if (fp32)
    hipLaunchKernelGGL(k_xpby_shift<float>, dim3(g), dim3(kBlock), 0, s, n, sc, inum, iden, sgn, imean, scale,
                       static_cast<const float*>(z), static_cast<float*>(p));
  else
    hipLaunchKernelGGL(k_xpby_shift<double>, dim3(g), dim3(kBlock), 0, s, n, sc, inum, iden, sgn, imean, scale,
                       static_cast<const double*>(z), static_cast<double*>(p));
  return hipGetLastError();
}

hipError_t launch_sum(bool fp32, int64_t n, const void* x, double* part, double* dst, hipStream_t s) {
  return launch_dot(fp32, n, x, nullptr, part, dst, s);
}

hipError_t launch_class_dot(bool fp32, int q, int N, const double* tab, const void* x, double* part,
                            int64_t part_cap, double* dst, hipStream_t s) {
  // one partial per (j, k) row
  if (static_cast<int64_t>(N) * N > part_cap) return hipErrorInvalidValue;
  ClassTab ct{};
  for (int i = 0; i < q * q * q; ++i) ct.v[i] = tab[i];
  if (fp32)
    hipLaunchKernelGGL(k_class_dot<float>, dim3(1, N, N), dim3(kBlock), 0, s, ct, q, N, static_cast<const float*>(x),
                       part);
  else
    hipLaunchKernelGGL(k_class_dot<double>, dim3(1, N, N), dim3(kBlock), 0, s, ct, q, N,
                       static_cast<const double*>(x), part);
  return launch_sum_partials(part, static_cast<int64_t>(N) * N, part_cap, dst, s);
}

hipError_t launch_sum_partials(const double* part, int64_t count, int64_t part_cap, double* dst, hipStream_t s) {
  // short runs: one block; long runs (N^2 row partials): fold chunks of 64 first,
  // into the tail of the partial buffer when it has room
  const int64_t chunk = 64;
  const int64_t blocks = (count + chunk - 1) / chunk;
  if (count <= 4 * kRedBlocks || count + blocks > part_cap || blocks > 65535) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kBlock), 0, s, part, static_cast<int>(count), dst);
    return hipGetLastError();
  }
  double* part2 = const_cast<double*>(part) + count;
  hipLaunchKernelGGL(k_fold, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, part, count, chunk, part2);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kBlock), 0, s, part2, static_cast<int>(blocks), dst);
  return hipGetLastError();
}

hipError_t launch_axpy2(bool fp32, int64_t n, const double* sc, int inum, int iden, void* u, const void* p, void* r,
                        const void* w, hipStream_t s) {
  const int g = grid_for(n);
  if (fp32)
    hipLaunchKernelGGL(k_axpy2<float>, dim3(g), dim3(kBlock), 0, s, n, sc, inum, iden, static_cast<float*>(u),
                       static_cast<const float*>(p), static_cast<float*>(r), static_cast<const float*>(w));
  else
    hipLaunchKernelGGL(k_axpy2<double>, dim3(g), dim3(kBlock), 0, s, n, sc, inum, iden, static_cast<double*>(u),
                       static_cast<const double*>(p), static_cast<double*>(r), static_cast<const double*>(w));
  return hipGetLastError();
}

hipError_t launch_xpby(bool fp32, int64_t n, const double* sc, int inum, int iden, double sgn, const void* z, void* p,
                       hipStream_t s) {
  const int g = grid_for(n);
  if (fp32)
    hipLaunchKernelGGL(k_xpby<float>, dim3(g), dim3(kBlock), 0, s, n, sc, inum, iden, sgn,
                       static_cast<const float*>(z), static_cast<float*>(p));
  else
    hipLaunchKernelGGL(k_xpby<double>, dim3(g), dim3(kBlock), 0, s, n, sc, inum, iden, sgn,
                       static_cast<const double*>(z), static_cast<double*>(p));
  return hipGetLastError();
}

hipError_t launch_shift(bool fp32, int64_t n, const double* sc, int i, double scale, void* v, hipStream_t s) {
  const int g = grid_for(n);
  if (fp32)
    hipLaunchKernelGGL(k_shift<float>, dim3(g), dim3(kBlock), 0, s, n, sc, i, scale, static_cast<float*>(v));
  else
    hipLaunchKernelGGL(k_shift<double>, dim3(g), dim3(kBlock), 0, s, n, sc, i, scale, static_cast<double*>(v));
  return hipGetLastError();
}

hipError_t launch_axpy(bool fp32, int64_t n, double a, const void* x, void* y, hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_axpy<float>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, a, static_cast<const float*>(x),
                       static_cast<float*>(y));
  else
    hipLaunchKernelGGL(k_axpy<double>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, a, static_cast<const double*>(x),
                       static_cast<double*>(y));
  return hipGetLastError();
}

hipError_t launch_class_axpy(bool fp32, int q, int N, const double* tab, double c, void* v, hipStream_t s) {
  ClassTab ct{};
  for (int i = 0; i < q * q * q; ++i) ct.v[i] = tab[i];
  if (fp32)
    hipLaunchKernelGGL(k_class_axpy<float>, class_grid(N), dim3(kBlock), 0, s, ct, q, N, c, static_cast<float*>(v));
  else
    hipLaunchKernelGGL(k_class_axpy<double>, class_grid(N), dim3(kBlock), 0, s, ct, q, N, c,
                       static_cast<double*>(v));
  return hipGetLastError();
}

hipError_t launch_splitmix_start(uint64_t key, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_splitmix_start, dim3(grid_for(n)), dim3(kBlock), 0, s, key, n, out);
  return hipGetLastError();
}

hipError_t launch_cast_d2f(int64_t n, const double* in, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_d2f, dim3(grid_for(n)), dim3(kBlock), 0, s, n, in, out);
  return hipGetLastError();
}

hipError_t launch_cast_f2d(int64_t n, const float* in, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_f2d, dim3(grid_for(n)), dim3(kBlock), 0, s, n, in, out);
  return hipGetLastError();
}

hipError_t launch_add_f2d(int64_t n, const float* c, double* u, hipStream_t s) {
  hipLaunchKernelGGL(k_add_f2d, dim3(grid_for(n)), dim3(kBlock), 0, s, n, c, u);
  return hipGetLastError();
}

hipError_t launch_fill_zero(bool fp32, int64_t n, void* v, hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_fill_zero<float>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, static_cast<float*>(v));
  else
    hipLaunchKernelGGL(k_fill_zero<double>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, static_cast<double*>(v));
  return hipGetLastError();
}

hipError_t launch_copy(bool fp32, int64_t n, const void* in, void* out, hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_copy<float>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, static_cast<const float*>(in),
                       static_cast<float*>(out));
  else
    hipLaunchKernelGGL(k_copy<double>, dim3(grid_for(n)), dim3(kBlock), 0, s, n, static_cast<const double*>(in),
                       static_cast<double*>(out));
  return hipGetLastError();
}

hipError_t launch_coarse(bool fp32, int n0, const double* ainv, const void* b, void* x, hipStream_t s) {
  if (n0 < 1 || n0 > kCoarseMax) return hipErrorInvalidValue;
  const dim3 grid((n0 + kCoarseRows - 1) / kCoarseRows);
  const size_t lds = sizeof(double) * static_cast<size_t>(n0);
  if (fp32)
    hipLaunchKernelGGL(k_coarse<float>, grid, dim3(64 * kCoarseRows), lds, s, n0, ainv,
                       static_cast<const float*>(b), static_cast<float*>(x));
  else
    hipLaunchKernelGGL(k_coarse<double>, grid, dim3(64 * kCoarseRows), lds, s, n0, ainv,
                       static_cast<const double*>(b), static_cast<double*>(x));
  return hipGetLastError();
}

}  // namespace gmg
