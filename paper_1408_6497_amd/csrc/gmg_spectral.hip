// Spectral FFT Poisson solve on a uniform periodic grid (Section 2.1): transform f,
// scale every Fourier coefficient by the inverse of the Laplacian's eigenvalue
// (a Hadamard product with 1 / (4 pi^2 |m|^2), m the integer wavevector in the
// band {-N/2 .. N/2-1}^3, and 0 for m = 0), transform back.
//
// The 3D transform is done here, without a library: five passes over an N^3 complex
// FP64 buffer, each a batch of 1D transforms of one axis.
//   1. x, forward, reading the real source f       (8 B in, 16 B out per point)
//   2. y, forward                                   (16 + 16)
//   3. z, forward, Hadamard scaling (with the 1/N^3 of the inverse), z inverse: the
//      whole z line is in LDS, so the scaling and the two z transforms cost one pass
//   4. y, inverse                                   (16 + 16)
//   5. x, inverse, writing the real part to u      (16 in, 8 out)
// 144 bytes of HBM traffic per point.
//
// One workgroup transforms kPts / N lines of one axis.  The lines go to LDS (padded
// by one value per line), then a Stockham autosort transform of radix 4 (and one
// radix-2 stage when log2 N is odd) runs in place in LDS: at each stage every thread
// reads its butterflies' inputs into registers, the block synchronises, and the
// outputs are written to their sorted positions.  For stage span Ns and radix R,
// butterfly j of a line reads points j + r N/R, multiplies point r by w^(r k N/(Ns R))
// with k = j mod Ns and w = exp(-2 pi i / N) (conjugated for the inverse), takes
// the R-point DFT and writes output r to (j div Ns) Ns R + k + r Ns.  The roots of
// unity come from a table of N values computed on the host in extended precision.
// Lines of the y and z passes are taken kPts / N consecutive in x, so a wavefront
// reads contiguous runs of x.
#include <cmath>
#include <vector>

#include "gmg_kernels.h"

namespace gmg {
namespace {

constexpr int kSpThreads = 256;
constexpr int kSpPts = 4096;  // points per workgroup (lines x N)

enum SpMode : int { kXFwdReal = 0, kYPass = 1, kZSolve = 2, kXInvReal = 3 };

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One Stockham stage of radix R on the lines in LDS (line stride NP values).
template <int R>
__device__ __forceinline__ void sp_stage(double2* data, const double2* __restrict__ tw, const int N, const int NP,
                                         const int Ns, const bool inv) {
  constexpr int B = kSpPts / (R * kSpThreads);  // butterflies per thread
  const int M = N / R;
  const int twstep = N / (Ns * R);
  double2 v[B][R];
  int dst[B];
#pragma unroll
  for (int u = 0; u < B; ++u) {
    const int b = threadIdx.x + u * kSpThreads;
    const int l = b / M, j = b - l * M;
    const int k = j % Ns;
    double2* line = data + l * NP;
#pragma unroll
    for (int r = 0; r < R; ++r) v[u][r] = line[j + r * M];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      double2 w = tw[(r * k * twstep) & (N - 1)];
      if (inv) w.y = -w.y;
      v[u][r] = cmul(v[u][r], w);
    }
    dst[u] = l * NP + (j / Ns) * Ns * R + k;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < B; ++u) {
    double2* o = data + dst[u];
    if constexpr (R == 4) {
      const double2 a = v[u][0], b = v[u][1], c = v[u][2], d = v[u][3];
      const double2 t0 = make_double2(a.x + c.x, a.y + c.y), t1 = make_double2(a.x - c.x, a.y - c.y);
      const double2 t2 = make_double2(b.x + d.x, b.y + d.y), t3 = make_double2(b.x - d.x, b.y - d.y);
      // forward: X1 = t1 - i t3, X3 = t1 + i t3; inverse: the signs of i swap
      const double2 it3 = inv ? make_double2(-t3.y, t3.x) : make_double2(t3.y, -t3.x);  // (+-i) t3
      o[0] = make_double2(t0.x + t2.x, t0.y + t2.y);
      o[Ns] = make_double2(t1.x + it3.x, t1.y + it3.y);
      o[2 * Ns] = make_double2(t0.x - t2.x, t0.y - t2.y);
      o[3 * Ns] = make_double2(t1.x - it3.x, t1.y - it3.y);
    } else {
      const double2 a = v[u][0], b = v[u][1];
      o[0] = make_double2(a.x + b.x, a.y + b.y);
      o[Ns] = make_double2(a.x - b.x, a.y - b.y);
    }
  }
  __syncthreads();
}

__device__ void sp_transform(double2* data, const double2* __restrict__ tw, const int N, const int NP, const bool inv) {
  for (int Ns = 1; Ns < N;) {
    if (N / Ns >= 4) {
      sp_stage<4>(data, tw, N, NP, Ns, inv);
      Ns *= 4;
    } else {
      sp_stage<2>(data, tw, N, NP, Ns, inv);
      Ns *= 2;
    }
  }
}

// Global offset of point a of line l for the pass's axis (0 x, 1 y, 2 z).
__device__ __forceinline__ int64_t sp_addr(const int axis, const int64_t l, const int a, const int N) {
  const int64_t n = N;
  if (axis == 0) return l * n + a;
  if (axis == 1) return (l % n) + n * a + n * n * (l / n);
  return l + n * n * a;
}

template <int MODE>
__global__ void __launch_bounds__(kSpThreads) k_spectral(const double* __restrict__ f, double2* buf,
                                                         const double2* __restrict__ tw, const int N,
                                                         double* __restrict__ u, const int inv_y) {
  extern __shared__ double2 data[];
  const int TX = kSpPts / N;  // lines per workgroup
  const int NP = N + 1;
  const int axis = (MODE == kXFwdReal || MODE == kXInvReal) ? 0 : (MODE == kYPass ? 1 : 2);
  const int64_t l0 = static_cast<int64_t>(blockIdx.x) * TX;
  // load: along the line for x (contiguous), across the lines for y and z (x-contiguous)
  for (int e = threadIdx.x; e < kSpPts; e += kSpThreads) {
    const int l = axis == 0 ? e / N : e % TX;
    const int a = axis == 0 ? e % N : e / TX;
    const int64_t g = sp_addr(axis, l0 + l, a, N);
    double2 v;
    if constexpr (MODE == kXFwdReal) v = make_double2(f[g], 0.0);
    else v = buf[g];
    data[l * NP + a] = v;
  }
  __syncthreads();
  if constexpr (MODE == kZSolve) {
    sp_transform(data, tw, N, NP, false);
    // Hadamard scaling: coefficient (mx, my, mz) of the transformed f over 4 pi^2 |m|^2,
    // with the 1/N^3 of the inverse transforms; the constant mode is set to 0
    const double norm = 1.0 / (4.0 * M_PI * M_PI * static_cast<double>(N) * N * N);
    for (int e = threadIdx.x; e < kSpPts; e += kSpThreads) {
      const int l = e / N, a = e % N;
      const int64_t lg = l0 + l;
      const int ix = static_cast<int>(lg % N), iy = static_cast<int>(lg / N);
      const int mx = ix < N / 2 ? ix : ix - N, my = iy < N / 2 ? iy : iy - N, mz = a < N / 2 ? a : a - N;
      const double mm = static_cast<double>(mx) * mx + static_cast<double>(my) * my + static_cast<double>(mz) * mz;
      const double s = mm > 0.0 ? norm / mm : 0.0;
      double2& d = data[l * NP + a];
      d.x *= s;
      d.y *= s;
    }
    __syncthreads();
    sp_transform(data, tw, N, NP, true);
  } else if constexpr (MODE == kYPass) {
    sp_transform(data, tw, N, NP, inv_y != 0);
  } else {
    sp_transform(data, tw, N, NP, MODE == kXInvReal);
  }
  for (int e = threadIdx.x; e < kSpPts; e += kSpThreads) {
    const int l = axis == 0 ? e / N : e % TX;
    const int a = axis == 0 ? e % N : e / TX;
    const int64_t g = sp_addr(axis, l0 + l, a, N);
    const double2 v = data[l * NP + a];
    if constexpr (MODE == kXInvReal) u[g] = v.x;
    else buf[g] = v;
  }
}

template <int MODE>
hipError_t sp_launch(const FftSpectral& s, const double* f, double* u, int inv_y, hipStream_t st) {
  const int N = s.N;
  const int64_t blocks = static_cast<int64_t>(N) * N * N / kSpPts;
  const size_t lds = sizeof(double2) * static_cast<size_t>(kSpPts / N) * (N + 1);
  hipLaunchKernelGGL(k_spectral<MODE>, dim3(static_cast<unsigned>(blocks)), dim3(kSpThreads), lds, st, f,
                     static_cast<double2*>(s.buf), static_cast<const double2*>(s.tw), N, u, inv_y);
  return hipGetLastError();
}

}  // namespace

FftSpectral::~FftSpectral() {
  if (buf) (void)hipFree(buf);
  if (tw) (void)hipFree(tw);
}

bool spectral_size_ok(int N) { return N >= 16 && N <= 1024 && (N & (N - 1)) == 0; }

hipError_t spectral_prepare(FftSpectral* s, int N) {
  if (!spectral_size_ok(N)) return hipErrorInvalidValue;
  if (s->N == N && s->buf && s->tw) return hipSuccess;
  if (s->buf) (void)hipFree(s->buf);
  if (s->tw) (void)hipFree(s->tw);
  s->buf = s->tw = nullptr;
  s->N = 0;
  std::vector<double2> w(N);
  const long double pi = std::acos(-1.0L);
  for (int k = 0; k < N; ++k) {
    const long double t = -2.0L * pi * k / N;
    w[k] = make_double2(static_cast<double>(std::cos(t)), static_cast<double>(std::sin(t)));
  }
  const size_t n3 = static_cast<size_t>(N) * N * N;
  if (hipMalloc(&s->buf, sizeof(double2) * n3) != hipSuccess || hipMalloc(&s->tw, sizeof(double2) * N) != hipSuccess) {
    if (s->buf) (void)hipFree(s->buf);
    if (s->tw) (void)hipFree(s->tw);
    s->buf = s->tw = nullptr;
    (void)hipGetLastError();
    return hipErrorOutOfMemory;
  }
  if (hipMemcpy(s->tw, w.data(), sizeof(double2) * N, hipMemcpyHostToDevice) != hipSuccess) return hipErrorUnknown;
  // tiles of up to 69.6 KB of LDS (4096 points plus one pad value per line)
  const int lds = static_cast<int>(sizeof(double2) * static_cast<size_t>(kSpPts / N) * (N + 1));
  const void* fns[4] = {reinterpret_cast<const void*>(&k_spectral<kXFwdReal>),
                        reinterpret_cast<const void*>(&k_spectral<kYPass>),
                        reinterpret_cast<const void*>(&k_spectral<kZSolve>),
                        reinterpret_cast<const void*>(&k_spectral<kXInvReal>)};
  for (const void* fn : fns) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
  }
  s->N = N;
  return hipSuccess;
}

hipError_t spectral_solve(const FftSpectral& s, const double* f, double* u, hipStream_t st) {
  if (!spectral_size_ok(s.N) || !s.buf || !s.tw) return hipErrorInvalidValue;
  hipError_t e = sp_launch<kXFwdReal>(s, f, nullptr, 0, st);
  if (e == hipSuccess) e = sp_launch<kYPass>(s, nullptr, nullptr, 0, st);
  if (e == hipSuccess) e = sp_launch<kZSolve>(s, nullptr, nullptr, 0, st);
  if (e == hipSuccess) e = sp_launch<kYPass>(s, nullptr, nullptr, 1, st);
  if (e == hipSuccess) e = sp_launch<kXInvReal>(s, nullptr, u, 0, st);
  return e;
}

}  // namespace gmg
