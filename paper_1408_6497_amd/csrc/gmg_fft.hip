// Exact solve of the uniform periodic Q1 system by the 3D FFT (the paper's uniform-grid
// FFT Poisson method of Section 2, applied to the same finite-element system the
// multigrid solves).
//
// On a uniform periodic mesh of N elements a side the Q1 matrix is
// A = K (x) M (x) M + M (x) K (x) M + M (x) M (x) K with the circulant 1D matrices
// K = circ(-1, 2, -1) / h and M = h circ(1, 4, 1) / 6, so the 3D Fourier modes are its
// eigenvectors, with eigenvalues
//   lambda(k) = kap(kx) mu(ky) mu(kz) + mu(kx) kap(ky) mu(kz) + mu(kx) mu(ky) kap(kz),
//   kap(k) = (2 - 2 cos(2 pi k / N)) / h,  mu(k) = h (4 + 2 cos(2 pi k / N)) / 6.
// u = F^-1 [ F(b) / lambda ] on the modes k != 0 and 0 on the constant mode (the solution
// of zero mean, which is the solution of zero integral for Q1 on a uniform mesh).
// hipFFT does the transforms (real-to-complex, FP64); the division runs here.
#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "gmg_kernels.h"
#include "gmg_setup_math.h"

namespace gmg {
namespace {

constexpr int kFftBlock = 256;

// spectrum layout of the real-to-complex transform: [kz][ky][kx], kx in [0, N/2]
__global__ void __launch_bounds__(kFftBlock) k_fft_q1_divide(hipfftDoubleComplex* spec, const int N, const double h) {
  const int NX = N / 2 + 1;
  const int64_t total = static_cast<int64_t>(N) * N * NX;
  const double norm = 1.0 / (static_cast<double>(N) * N * N);
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int kx = static_cast<int>(t % NX);
    const int ky = static_cast<int>((t / NX) % N);
    const int kz = static_cast<int>(t / (static_cast<int64_t>(NX) * N));
    const double cx = cospi(2.0 * kx / N), cy = cospi(2.0 * ky / N), cz = cospi(2.0 * kz / N);
    const double ax = (2.0 - 2.0 * cx) / h, ay = (2.0 - 2.0 * cy) / h, az = (2.0 - 2.0 * cz) / h;
    const double mx = h * (4.0 + 2.0 * cx) / 6.0, my = h * (4.0 + 2.0 * cy) / 6.0, mz = h * (4.0 + 2.0 * cz) / 6.0;
    const double lam = ax * my * mz + mx * ay * mz + mx * my * az;
    const double s = (kx == 0 && ky == 0 && kz == 0) ? 0.0 : norm / lam;
    spec[t].x *= s;
    spec[t].y *= s;
  }
}

}  // namespace

static inline hipfftHandle fft_handle(void* p) { return static_cast<hipfftHandle>(p); }

// Plans and buffers of one FFT object are released together, so that a prepare that
// fails half way (or one for another size) leaves nothing behind and starts afresh.
template <typename F>
void fft_release(F* f) {
  if (f->fwd_ok) (void)hipfftDestroy(fft_handle(f->fwd));
  if (f->inv_ok) (void)hipfftDestroy(fft_handle(f->inv));
  f->fwd_ok = f->inv_ok = false;
  f->fwd = f->inv = nullptr;
  if (f->spec) (void)hipFree(f->spec);
  f->spec = nullptr;
}

FftQ1::~FftQ1() { fft_release(this); }

hipError_t fft_q1_prepare(FftQ1* f, int N) {
  if (f->N == N && f->fwd_ok && f->inv_ok && f->spec) return hipSuccess;
  if (N < 2) return hipErrorInvalidValue;
  fft_release(f);
  f->N = 0;
  const size_t bytes = sizeof(hipfftDoubleComplex) * static_cast<size_t>(N) * N * (N / 2 + 1);
  hipError_t e = hipMalloc(&f->spec, bytes);
  if (e != hipSuccess) {
    f->spec = nullptr;
    return e;
  }
  hipfftHandle h = nullptr;
  if (hipfftPlan3d(&h, N, N, N, HIPFFT_D2Z) != HIPFFT_SUCCESS) {
    fft_release(f);
    return hipErrorUnknown;
  }
  f->fwd = h;
  f->fwd_ok = true;
  if (hipfftPlan3d(&h, N, N, N, HIPFFT_Z2D) != HIPFFT_SUCCESS) {
    fft_release(f);
    return hipErrorUnknown;
  }
  f->inv = h;
  f->inv_ok = true;
  f->N = N;
  return hipSuccess;
}

hipError_t fft_q1_solve(FftQ1* f, const double* b, double* u, hipStream_t s) {
  const int N = f->N;
  const size_t n3 = static_cast<size_t>(N) * N * N;
  // the transforms read u, never b (a complex-to-real transform may overwrite its input)
  hipError_t e = hipMemcpyAsync(u, b, sizeof(double) * n3, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  if (hipfftSetStream(fft_handle(f->fwd), s) != HIPFFT_SUCCESS || hipfftSetStream(fft_handle(f->inv), s) != HIPFFT_SUCCESS)
    return hipErrorUnknown;
  if (hipfftExecD2Z(fft_handle(f->fwd), u, static_cast<hipfftDoubleComplex*>(f->spec)) != HIPFFT_SUCCESS)
    return hipErrorUnknown;
  const int64_t total = static_cast<int64_t>(N) * N * (N / 2 + 1);
  int64_t g = (total + kFftBlock - 1) / kFftBlock;
  if (g > 65535) g = 65535;
  hipLaunchKernelGGL(k_fft_q1_divide, dim3(static_cast<unsigned>(g)), dim3(kFftBlock), 0, s,
                     static_cast<hipfftDoubleComplex*>(f->spec), N, 1.0 / N);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (hipfftExecZ2D(fft_handle(f->inv), static_cast<hipfftDoubleComplex*>(f->spec), u) != HIPFFT_SUCCESS)
    return hipErrorUnknown;
  return hipSuccess;
}

}  // namespace gmg

// ---------------------------------------------------------------------------------------
// Q2: the two node classes per axis (vertex, midpoint) make each 1D matrix block-circulant
// over the elements, with the 2x2 Hermitian symbol P(t)^H E P(t) of the element matrix E
// (P maps a cell's (vertex, midpoint) to the element's nodes v_e, m_e, v_{e+1} = e^{it} v_e).
// Per axis and wavenumber the pencil (K, M) has M-orthonormal eigenvectors V (V^H M V = I,
// V^H K V = diag(lam)); the 3D matrix is then diagonalised by W = Vx (x) Vy (x) Vz with
// eigenvalues lam_x + lam_y + lam_z, so A^-1 = W diag(1 / (lam_x + lam_y + lam_z)) W^H on the
// class spectra.  The zero eigenvalue (t = 0 on every axis, the constant) has the
// M-weighted coefficient of u, its integral, which is set to 0.
namespace gmg {
namespace {

struct Axis2 {
  double vr[2][2], vi[2][2];  // V (rows: class, columns: mode)
  double lam[2];
};

__global__ void __launch_bounds__(kFftBlock) k_split_classes(const double* __restrict__ b, double* __restrict__ bc,
                                                              const int n) {
  const int N = 2 * n;
  const int64_t n3 = static_cast<int64_t>(n) * n * n;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < 8 * n3;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int c = static_cast<int>(t / n3);
    const int64_t e = t - c * n3;
    const int ex = static_cast<int>(e % n), ey = static_cast<int>((e / n) % n), ez = static_cast<int>(e / (int64_t(n) * n));
    const int i = 2 * ex + (c & 1), j = 2 * ey + ((c >> 1) & 1), k = 2 * ez + (c >> 2);
    bc[t] = b[(static_cast<int64_t>(k) * N + j) * N + i];
  }
}

__global__ void __launch_bounds__(kFftBlock) k_merge_classes(const double* __restrict__ uc, double* __restrict__ u,
                                                              const int n) {
  const int N = 2 * n;
  const int64_t n3 = static_cast<int64_t>(n) * n * n;
  const double norm = 1.0 / static_cast<double>(n3);
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < 8 * n3;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int c = static_cast<int>(t / n3);
    const int64_t e = t - c * n3;
    const int ex = static_cast<int>(e % n), ey = static_cast<int>((e / n) % n), ez = static_cast<int>(e / (int64_t(n) * n));
    const int i = 2 * ex + (c & 1), j = 2 * ey + ((c >> 1) & 1), k = 2 * ez + (c >> 2);
    u[(static_cast<int64_t>(k) * N + j) * N + i] = uc[t] * norm;
  }
}

// y = op(V) x along one axis of the 2x2x2 block (op = V^H when herm), complex
__device__ __forceinline__ void axis_apply(const Axis2& a, bool herm, int axis, double (&xr)[8], double (&xi)[8]) {
  const int stride = 1 << axis;
#pragma unroll
  for (int base = 0; base < 8; ++base) {
    if (base & stride) continue;
    const double r0 = xr[base], i0 = xi[base], r1 = xr[base + stride], i1 = xi[base + stride];
    double yr[2], yi[2];
#pragma unroll
    for (int o = 0; o < 2; ++o) {
      // herm: y_o = sum_c conj(V[c][o]) x_c ; else: y_o = sum_m V[o][m] x_m
      const double ar = herm ? a.vr[0][o] : a.vr[o][0], ai = herm ? -a.vi[0][o] : a.vi[o][0];
      const double br = herm ? a.vr[1][o] : a.vr[o][1], bi = herm ? -a.vi[1][o] : a.vi[o][1];
      yr[o] = ar * r0 - ai * i0 + br * r1 - bi * i1;
      yi[o] = ar * i0 + ai * r0 + br * i1 + bi * r1;
    }
    xr[base] = yr[0];
    xi[base] = yi[0];
    xr[base + stride] = yr[1];
    xi[base + stride] = yi[1];
  }
}

// spectra [8 classes][kz][ky][kx], kx in [0, n/2]
__global__ void __launch_bounds__(kFftBlock) k_fft_q2_solve(hipfftDoubleComplex* spec, const Axis2* __restrict__ ax,
                                                             const int n) {
  const int NX = n / 2 + 1;
  const int64_t m = static_cast<int64_t>(n) * n * NX;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < m;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int kx = static_cast<int>(t % NX);
    const int ky = static_cast<int>((t / NX) % n);
    const int kz = static_cast<int>(t / (static_cast<int64_t>(NX) * n));
    double xr[8], xi[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      xr[c] = spec[c * m + t].x;
      xi[c] = spec[c * m + t].y;
    }
    const Axis2 X = ax[kx], Y = ax[ky], Z = ax[kz];
    axis_apply(X, true, 0, xr, xi);
    axis_apply(Y, true, 1, xr, xi);
    axis_apply(Z, true, 2, xr, xi);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double lam = X.lam[c & 1] + Y.lam[(c >> 1) & 1] + Z.lam[c >> 2];
      const double s = lam > 0.0 ? 1.0 / lam : 0.0;  // the constant mode: 0
      xr[c] *= s;
      xi[c] *= s;
    }
    axis_apply(Z, false, 2, xr, xi);
    axis_apply(Y, false, 1, xr, xi);
    axis_apply(X, false, 0, xr, xi);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      spec[c * m + t].x = xr[c];
      spec[c * m + t].y = xi[c];
    }
  }
}

}  // namespace

// the class-split objects (Q2, Q4) also hold the class arrays and the axis tables
template <typename F>
void fft_release_classes(F* f) {
  fft_release(f);
  if (f->cls) (void)hipFree(f->cls);
  if (f->axis) (void)hipFree(f->axis);
  f->cls = f->axis = nullptr;
  f->n = 0;
}

FftQ2::~FftQ2() { fft_release_classes(this); }

// 1D symbols of the Q2 element matrices (LGL nodes 0, 1/2, 1 on an element of width h) and
// the M-orthonormal eigenvectors of each 2x2 pencil, for the n wavenumbers t = 2 pi k / n:
// lam from det(K - lam M) = 0, each eigenvector from a row of K - lam M, scaled to
// v^H M v = 1 (eigenvectors of distinct eigenvalues are M-orthogonal).
static void q2_axis_tables(int n, std::vector<Axis2>* out) {
  const double h = 1.0 / n;
  const double k3[3][3] = {{7.0 / 3, -8.0 / 3, 1.0 / 3}, {-8.0 / 3, 16.0 / 3, -8.0 / 3}, {1.0 / 3, -8.0 / 3, 7.0 / 3}};
  const double m3[3][3] = {{4.0 / 30, 2.0 / 30, -1.0 / 30}, {2.0 / 30, 16.0 / 30, 2.0 / 30}, {-1.0 / 30, 2.0 / 30, 4.0 / 30}};
  out->resize(n);
  for (int k = 0; k < n; ++k) {
    const double t = 2.0 * M_PI * k / n, ct = std::cos(t), st = std::sin(t);
    // S = P^H E P: S00 = E00 + E22 + 2 E02 cos t, S01 = E01 + E21 e^{-it}, S11 = E11
    auto sym = [&](const double (&E)[3][3], double s, double* a, double* br, double* bi, double* d) {
      *a = s * (E[0][0] + E[2][2] + 2.0 * E[0][2] * ct);
      *br = s * (E[0][1] + E[2][1] * ct);
      *bi = s * (-E[2][1] * st);
      *d = s * E[1][1];
    };
    double ka, kbr, kbi, kd, ma, mbr, mbi, md;
    sym(k3, 1.0 / h, &ka, &kbr, &kbi, &kd);
    sym(m3, h, &ma, &mbr, &mbi, &md);
    // det(K - lam M) = qa lam^2 + qb lam + qc.  det K = ka kd - |kb|^2 vanishes like t^2,
    // so it is taken in closed form: with the Q2 rows above, ka kd - |kb|^2 =
    // (32/3)(1 - cos t) / h^2 = (64/3) sin^2(t/2) / h^2, and the small root as
    // 2 qc / (-qb + disc) (qa > 0, qb < 0), so neither loses digits to cancellation
    // as t -> 0.
    const double qa = ma * md - (mbr * mbr + mbi * mbi);
    const double qb = -(ka * md + kd * ma) + 2.0 * (kbr * mbr + kbi * mbi);
    const double sh = std::sin(0.5 * t);
    const double qc = (64.0 / 3.0) * sh * sh / (h * h);
    const double disc = std::sqrt(std::max(0.0, qb * qb - 4.0 * qa * qc));
    Axis2& A = (*out)[k];
    A.lam[0] = 2.0 * qc / (-qb + disc);
    A.lam[1] = (-qb + disc) / (2.0 * qa);
    if (k == 0) A.lam[0] = 0.0;  // the constant is exactly in the kernel of K at t = 0
    for (int o = 0; o < 2; ++o) {
      const double lam = A.lam[o];
      // row 0 of K - lam M: (a0) v0 + (b0) v1 = 0 -> v = (b0, -a0); row 1: v = (d1, -c1)
      const double a0 = ka - lam * ma, b0r = kbr - lam * mbr, b0i = kbi - lam * mbi;
      const double c1r = kbr - lam * mbr, c1i = -(kbi - lam * mbi), d1 = kd - lam * md;
      double v0r = b0r, v0i = b0i, v1r = -a0, v1i = 0.0;
      double nn = v0r * v0r + v0i * v0i + v1r * v1r;
      const double w0r = d1, w0i = 0.0, w1r = -c1r, w1i = -c1i;
      const double nn2 = w0r * w0r + w1r * w1r + w1i * w1i;
      if (nn2 > nn) {
        v0r = w0r; v0i = w0i; v1r = w1r; v1i = w1i; nn = nn2;
      }
      if (o == 1 && disc <= 1e-14 * std::fabs(qb)) {  // a double eigenvalue: M-orthogonalise e2
        v0r = 0.0; v0i = 0.0; v1r = 1.0; v1i = 0.0;
        // v <- v - (u^H M v) u with u = column 0
        const double u0r = A.vr[0][0], u0i = A.vi[0][0], u1r = A.vr[1][0], u1i = A.vi[1][0];
        // M v = (ma v0 + mb v1, conj(mb) v0 + md v1) with v = e2: (mb, md)
        const double mvr0 = mbr, mvi0 = mbi, mvr1 = md, mvi1 = 0.0;
        const double pr = u0r * mvr0 + u0i * mvi0 + u1r * mvr1 + u1i * mvi1;  // Re(u^H M v)
        const double pi = u0r * mvi0 - u0i * mvr0 + u1r * mvi1 - u1i * mvr1;  // Im(u^H M v)
        v0r -= pr * u0r - pi * u0i; v0i -= pr * u0i + pi * u0r;
        v1r -= pr * u1r - pi * u1i; v1i -= pr * u1i + pi * u1r;
      } else if (nn <= 1e-300) {
        v0r = o == 0 ? 1.0 : 0.0; v1r = o == 0 ? 0.0 : 1.0; v0i = v1i = 0.0;
      }
      // scale to v^H M v = 1: v^H M v = ma |v0|^2 + md |v1|^2 + 2 Re(conj(v0) mb v1)
      const double mb_v1r = mbr * v1r - mbi * v1i, mb_v1i = mbr * v1i + mbi * v1r;
      const double vmv = ma * (v0r * v0r + v0i * v0i) + md * (v1r * v1r + v1i * v1i) +
                         2.0 * (v0r * mb_v1r + v0i * mb_v1i);
      const double sc = 1.0 / std::sqrt(vmv);
      A.vr[0][o] = v0r * sc; A.vi[0][o] = v0i * sc; A.vr[1][o] = v1r * sc; A.vi[1][o] = v1i * sc;
    }
  }
}

// Buffers, axis tables and batched plans of a class-split solve with NC classes; on any
// failure everything made so far is released and f->n stays 0.
template <typename F, typename Tab>
hipError_t fft_prepare_classes(F* f, int n, int NC, const std::vector<Tab>& tab) {
  fft_release_classes(f);
  const size_t n3 = static_cast<size_t>(n) * n * n;
  const size_t m = static_cast<size_t>(n) * n * (n / 2 + 1);
  hipError_t e = hipSuccess;
  if (hipMalloc(&f->spec, sizeof(hipfftDoubleComplex) * NC * m) != hipSuccess ||
      hipMalloc(&f->cls, sizeof(double) * NC * n3) != hipSuccess ||
      hipMalloc(&f->axis, sizeof(Tab) * n) != hipSuccess)
    e = hipErrorOutOfMemory;
  if (e == hipSuccess && hipMemcpy(f->axis, tab.data(), sizeof(Tab) * n, hipMemcpyHostToDevice) != hipSuccess)
    e = hipErrorUnknown;
  int dims[3] = {n, n, n};
  hipfftHandle h = nullptr;
  if (e == hipSuccess) {
    if (hipfftPlanMany(&h, 3, dims, nullptr, 1, static_cast<int>(n3), nullptr, 1, static_cast<int>(m), HIPFFT_D2Z,
                       NC) == HIPFFT_SUCCESS) {
      f->fwd = h;
      f->fwd_ok = true;
    } else {
      e = hipErrorUnknown;
    }
  }
  if (e == hipSuccess) {
    if (hipfftPlanMany(&h, 3, dims, nullptr, 1, static_cast<int>(m), nullptr, 1, static_cast<int>(n3), HIPFFT_Z2D,
                       NC) == HIPFFT_SUCCESS) {
      f->inv = h;
      f->inv_ok = true;
    } else {
      e = hipErrorUnknown;
    }
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fft_release_classes(f);
    return e;
  }
  f->n = n;
  return hipSuccess;
}

hipError_t fft_q2_prepare(FftQ2* f, int n) {
  if (f->n == n && f->fwd_ok && f->inv_ok && f->spec) return hipSuccess;
  if (n < 2 || (n & 1)) return hipErrorInvalidValue;
  std::vector<Axis2> tab;
  q2_axis_tables(n, &tab);
  return fft_prepare_classes(f, n, 8, tab);
}

hipError_t fft_q2_solve(FftQ2* f, const double* b, double* u, hipStream_t s) {
  const int n = f->n;
  const int64_t total = 8 * static_cast<int64_t>(n) * n * n;
  int64_t g = (total + kFftBlock - 1) / kFftBlock;
  if (g > 65535) g = 65535;
  hipLaunchKernelGGL(k_split_classes, dim3(static_cast<unsigned>(g)), dim3(kFftBlock), 0, s, b,
                     static_cast<double*>(f->cls), n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (hipfftSetStream(fft_handle(f->fwd), s) != HIPFFT_SUCCESS || hipfftSetStream(fft_handle(f->inv), s) != HIPFFT_SUCCESS)
    return hipErrorUnknown;
  if (hipfftExecD2Z(fft_handle(f->fwd), static_cast<double*>(f->cls), static_cast<hipfftDoubleComplex*>(f->spec)) !=
      HIPFFT_SUCCESS)
    return hipErrorUnknown;
  const int64_t m = static_cast<int64_t>(n) * n * (n / 2 + 1);
  int64_t g2 = (m + kFftBlock - 1) / kFftBlock;
  if (g2 > 65535) g2 = 65535;
  hipLaunchKernelGGL(k_fft_q2_solve, dim3(static_cast<unsigned>(g2)), dim3(kFftBlock), 0, s,
                     static_cast<hipfftDoubleComplex*>(f->spec), static_cast<const Axis2*>(f->axis), n);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (hipfftExecZ2D(fft_handle(f->inv), static_cast<hipfftDoubleComplex*>(f->spec), static_cast<double*>(f->cls)) !=
      HIPFFT_SUCCESS)
    return hipErrorUnknown;
  hipLaunchKernelGGL(k_merge_classes, dim3(static_cast<unsigned>(g)), dim3(kFftBlock), 0, s,
                     static_cast<const double*>(f->cls), u, n);
  return hipGetLastError();
}

}  // namespace gmg

// ---------------------------------------------------------------------------------------
// Q4: the same construction with 4 node classes per axis (64 per element cell) and 4x4
// pencils, whose M-orthonormal eigenbases come from a Cholesky factor of M and a Jacobi
// eigen-decomposition of L^-1 K L^-H (through its real symmetric 2q x 2q embedding).
namespace gmg {
namespace {

template <int Q>
struct AxisQ {
  double vr[Q][Q], vi[Q][Q];  // V (rows: class, columns: mode)
  double lam[Q];
};

template <int Q>
__global__ void __launch_bounds__(kFftBlock) k_split_q(const double* __restrict__ b, double* __restrict__ bc, const int n,
                                                       const int merge) {
  constexpr int NC = Q * Q * Q;
  const int N = Q * n;
  const int64_t n3 = static_cast<int64_t>(n) * n * n;
  const double norm = 1.0 / static_cast<double>(n3);
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < NC * n3;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int c = static_cast<int>(t / n3);
    const int64_t e = t - c * n3;
    const int ex = static_cast<int>(e % n), ey = static_cast<int>((e / n) % n), ez = static_cast<int>(e / (int64_t(n) * n));
    const int i = Q * ex + c % Q, j = Q * ey + (c / Q) % Q, k = Q * ez + c / (Q * Q);
    const int64_t idx = (static_cast<int64_t>(k) * N + j) * N + i;
    if (merge) const_cast<double*>(b)[idx] = bc[t] * norm;
    else bc[t] = b[idx];
  }
}

template <int Q>
__device__ __forceinline__ void axis_apply_q(const AxisQ<Q>& a, bool herm, int stride, double (&xr)[Q * Q * Q],
                                             double (&xi)[Q * Q * Q]) {
  constexpr int NC = Q * Q * Q;
#pragma unroll
  for (int base = 0; base < NC; ++base) {
    if ((base / stride) % Q != 0) continue;
    double yr[Q], yi[Q];
#pragma unroll
    for (int o = 0; o < Q; ++o) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int m = 0; m < Q; ++m) {
        const double ar = herm ? a.vr[m][o] : a.vr[o][m];
        const double ai = herm ? -a.vi[m][o] : a.vi[o][m];
        const double xrr = xr[base + m * stride], xii = xi[base + m * stride];
        sr += ar * xrr - ai * xii;
        si += ar * xii + ai * xrr;
      }
      yr[o] = sr;
      yi[o] = si;
    }
#pragma unroll
    for (int o = 0; o < Q; ++o) {
      xr[base + o * stride] = yr[o];
      xi[base + o * stride] = yi[o];
    }
  }
}

template <int Q>
__global__ void __launch_bounds__(kFftBlock) k_fft_solve_q(hipfftDoubleComplex* spec, const AxisQ<Q>* __restrict__ ax,
                                                           const int n) {
  constexpr int NC = Q * Q * Q;
  const int NX = n / 2 + 1;
  const int64_t m = static_cast<int64_t>(n) * n * NX;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < m;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int kx = static_cast<int>(t % NX);
    const int ky = static_cast<int>((t / NX) % n);
    const int kz = static_cast<int>(t / (static_cast<int64_t>(NX) * n));
    double xr[NC], xi[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      xr[c] = spec[c * m + t].x;
      xi[c] = spec[c * m + t].y;
    }
    axis_apply_q<Q>(ax[kx], true, 1, xr, xi);
    axis_apply_q<Q>(ax[ky], true, Q, xr, xi);
    axis_apply_q<Q>(ax[kz], true, Q * Q, xr, xi);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double lam = ax[kx].lam[c % Q] + ax[ky].lam[(c / Q) % Q] + ax[kz].lam[c / (Q * Q)];
      const double s = lam > 0.0 ? 1.0 / lam : 0.0;  // the constant mode: 0
      xr[c] *= s;
      xi[c] *= s;
    }
    axis_apply_q<Q>(ax[kz], false, Q * Q, xr, xi);
    axis_apply_q<Q>(ax[ky], false, Q, xr, xi);
    axis_apply_q<Q>(ax[kx], false, 1, xr, xi);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      spec[c * m + t].x = xr[c];
      spec[c * m + t].y = xi[c];
    }
  }
}

// Eigen-decomposition of a real symmetric matrix (cyclic Jacobi), ascending eigenvalues,
// eigenvectors as the columns of v (row-major, dimension d).
template <typename R>
void jacobi_eigen(int d, std::vector<R> a, std::vector<R>* w, std::vector<R>* v) {
  using std::fabs;
  using std::sqrt;
  v->assign(static_cast<size_t>(d) * d, 0.0);
  for (int i = 0; i < d; ++i) (*v)[i * d + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    R off = 0, tot = 0;
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        tot += a[i * d + j] * a[i * d + j];
        if (i != j) off += a[i * d + j] * a[i * d + j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < d; ++p)
      for (int r = p + 1; r < d; ++r) {
        const R apr = a[p * d + r];
        if (fabs(apr) < R(1e-300)) continue;
        const R theta = (a[r * d + r] - a[p * d + p]) / (2 * apr);
        const R t = (theta >= 0 ? R(1) : R(-1)) / (fabs(theta) + sqrt(theta * theta + 1));
        const R c = 1 / sqrt(t * t + 1), s = t * c;
        for (int k = 0; k < d; ++k) {  // columns p, r
          const R akp = a[k * d + p], akr = a[k * d + r];
          a[k * d + p] = c * akp - s * akr;
          a[k * d + r] = s * akp + c * akr;
        }
        for (int k = 0; k < d; ++k) {  // rows p, r
          const R apk = a[p * d + k], ark = a[r * d + k];
          a[p * d + k] = c * apk - s * ark;
          a[r * d + k] = s * apk + c * ark;
        }
        for (int k = 0; k < d; ++k) {
          const R vkp = (*v)[k * d + p], vkr = (*v)[k * d + r];
          (*v)[k * d + p] = c * vkp - s * vkr;
          (*v)[k * d + r] = s * vkp + c * vkr;
        }
      }
  }
  std::vector<int> ord(d);
  for (int i = 0; i < d; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int x, int y) { return a[x * d + x] < a[y * d + y]; });
  std::vector<R> vs(static_cast<size_t>(d) * d);
  w->resize(d);
  for (int j = 0; j < d; ++j) {
    (*w)[j] = a[ord[j] * d + ord[j]];
    for (int k = 0; k < d; ++k) vs[k * d + j] = (*v)[k * d + ord[j]];
  }
  *v = vs;
}

// The tables are computed in x87 extended precision (64-bit significand) and rounded to
// FP64 at the end: the smallest eigenvalue of a pencil vanishes like t^2 at small
// wavenumbers t while the symbol's entries stay O(1/h), so an FP64 computation would
// lose about log10(1/t^2) digits of it (3 at n = 256); 11 more bits keep it at FP64
// accuracy up to the largest supported n.
template <int Q>
void axis_tables_q(int n, std::vector<AxisQ<Q>>* out) {
  using R = long double;
  using C = std::complex<R>;
  std::vector<double> khat64, mhat;
  reference_matrices(Q, &khat64, &mhat);
  const int p = Q + 1;
  // The stiffness rows sum to zero (the derivative of a constant vanishes); the FP64 table
  // does so only to rounding, which would put an O(eps / h) eigenvalue error at every small
  // wavenumber.  The diagonal is set to minus the row's off-diagonal sum in extended
  // precision, so the constant is exactly in the kernel at t = 0 and the small branch
  // vanishes like t^2 without an eps floor.
  std::vector<R> khat(khat64.begin(), khat64.end());
  for (int a = 0; a <= Q; ++a) {
    R off = 0;
    for (int b = 0; b <= Q; ++b)
      if (b != a) off += khat[a * p + b];
    khat[a * p + a] = -off;
  }
  const R h = R(1) / n;
  const R pi = std::acos(R(-1));
  out->resize(n);
  for (int k = 0; k < n; ++k) {
    const C ph = std::polar(R(1), 2 * pi * k / n);
    // S = P^H E P, P: class a -> local node a (a < q), and local node q = e^{it} class 0
    auto sym = [&](const auto& E, R sc, C (&S)[Q][Q]) {
      for (int a = 0; a < Q; ++a)
        for (int b = 0; b < Q; ++b) {
          C s = R(E[a * p + b]);
          if (a == 0) s += std::conj(ph) * R(E[Q * p + b]);
          if (b == 0) s += R(E[a * p + Q]) * ph;
          if (a == 0 && b == 0) s += R(E[Q * p + Q]);
          S[a][b] = sc * s;
        }
    };
    C K[Q][Q], M[Q][Q], L[Q][Q] = {}, Li[Q][Q] = {};
    sym(khat, 1 / h, K);
    sym(mhat, h, M);
    for (int j = 0; j < Q; ++j) {  // Cholesky M = L L^H
      C s = M[j][j];
      for (int t = 0; t < j; ++t) s -= L[j][t] * std::conj(L[j][t]);
      L[j][j] = std::sqrt(s.real());
      for (int i = j + 1; i < Q; ++i) {
        C u = M[i][j];
        for (int t = 0; t < j; ++t) u -= L[i][t] * std::conj(L[j][t]);
        L[i][j] = u / L[j][j];
      }
    }
    for (int j = 0; j < Q; ++j) {  // L^-1 by forward substitution
      Li[j][j] = R(1) / L[j][j];
      for (int i = j + 1; i < Q; ++i) {
        C s = 0;
        for (int t = j; t < i; ++t) s += L[i][t] * Li[t][j];
        Li[i][j] = -s / L[i][i];
      }
    }
    C Cm[Q][Q];  // L^-1 K L^-H
    for (int i = 0; i < Q; ++i)
      for (int j = 0; j < Q; ++j) {
        C s = 0;
        for (int a = 0; a < Q; ++a)
          for (int b = 0; b < Q; ++b) s += Li[i][a] * K[a][b] * std::conj(Li[j][b]);
        Cm[i][j] = s;
      }
    // real symmetric embedding [[Re, -Im], [Im, Re]]: every eigenvalue twice
    const int d = 2 * Q;
    std::vector<R> Re(static_cast<size_t>(d) * d), w, v;
    for (int i = 0; i < Q; ++i)
      for (int j = 0; j < Q; ++j) {
        Re[i * d + j] = Cm[i][j].real();
        Re[i * d + Q + j] = -Cm[i][j].imag();
        Re[(Q + i) * d + j] = Cm[i][j].imag();
        Re[(Q + i) * d + Q + j] = Cm[i][j].real();
      }
    jacobi_eigen<R>(d, Re, &w, &v);
    // complex eigenvectors z = y_re + i y_im from the real ones, kept when independent of
    // those already taken (Gram-Schmidt), in ascending eigenvalue order
    std::vector<std::vector<C>> Z;
    std::vector<R> lam;
    for (int j = 0; j < d && static_cast<int>(Z.size()) < Q; ++j) {
      std::vector<C> z(Q);
      for (int i = 0; i < Q; ++i) z[i] = C(v[i * d + j], v[(Q + i) * d + j]);
      for (const auto& y : Z) {
        C dot = 0;
        for (int i = 0; i < Q; ++i) dot += std::conj(y[i]) * z[i];
        for (int i = 0; i < Q; ++i) z[i] -= dot * y[i];
      }
      R nn = 0;
      for (int i = 0; i < Q; ++i) nn += std::norm(z[i]);
      if (nn < R(1e-12)) continue;
      for (int i = 0; i < Q; ++i) z[i] /= std::sqrt(nn);
      Z.push_back(z);
      lam.push_back(w[j]);
    }
    AxisQ<Q>& A = (*out)[k];
    for (int o = 0; o < Q; ++o) {
      A.lam[o] = o < static_cast<int>(lam.size()) ? static_cast<double>(lam[o]) : 0.0;
      for (int r = 0; r < Q; ++r) {  // V = L^-H Z: (L^-H)[r][i] = conj(Li[i][r])
        C s = 0;
        if (o < static_cast<int>(Z.size()))
          for (int i = 0; i < Q; ++i) s += std::conj(Li[i][r]) * Z[o][i];
        A.vr[r][o] = static_cast<double>(s.real());
        A.vi[r][o] = static_cast<double>(s.imag());
      }
    }
    if (k == 0) A.lam[0] = 0.0;  // the constant is exactly in the kernel of K at t = 0
  }
}

}  // namespace

FftQ4::~FftQ4() { fft_release_classes(this); }

hipError_t fft_q4_prepare(FftQ4* f, int n) {
  if (f->n == n && f->fwd_ok && f->inv_ok && f->spec) return hipSuccess;
  if (n < 2) return hipErrorInvalidValue;
  std::vector<AxisQ<4>> tab;
  axis_tables_q<4>(n, &tab);
  return fft_prepare_classes(f, n, 64, tab);
}

hipError_t fft_q4_solve(FftQ4* f, const double* b, double* u, hipStream_t s) {
  const int n = f->n;
  const int64_t total = 64 * static_cast<int64_t>(n) * n * n;
  int64_t g = (total + kFftBlock - 1) / kFftBlock;
  if (g > 65535) g = 65535;
  hipLaunchKernelGGL(k_split_q<4>, dim3(static_cast<unsigned>(g)), dim3(kFftBlock), 0, s, b,
                     static_cast<double*>(f->cls), n, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (hipfftSetStream(fft_handle(f->fwd), s) != HIPFFT_SUCCESS || hipfftSetStream(fft_handle(f->inv), s) != HIPFFT_SUCCESS)
    return hipErrorUnknown;
  if (hipfftExecD2Z(fft_handle(f->fwd), static_cast<double*>(f->cls), static_cast<hipfftDoubleComplex*>(f->spec)) !=
      HIPFFT_SUCCESS)
    return hipErrorUnknown;
  const int64_t m = static_cast<int64_t>(n) * n * (n / 2 + 1);
  int64_t g2 = (m + kFftBlock - 1) / kFftBlock;
  if (g2 > 65535) g2 = 65535;
  hipLaunchKernelGGL(k_fft_solve_q<4>, dim3(static_cast<unsigned>(g2)), dim3(kFftBlock), 0, s,
                     static_cast<hipfftDoubleComplex*>(f->spec), static_cast<const AxisQ<4>*>(f->axis), n);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (hipfftExecZ2D(fft_handle(f->inv), static_cast<hipfftDoubleComplex*>(f->spec), static_cast<double*>(f->cls)) !=
      HIPFFT_SUCCESS)
    return hipErrorUnknown;
  hipLaunchKernelGGL(k_split_q<4>, dim3(static_cast<unsigned>(g)), dim3(kFftBlock), 0, s, u,
                     static_cast<double*>(f->cls), n, 1);
  return hipGetLastError();
}

}  // namespace gmg
