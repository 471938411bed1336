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
#include <vector>

#include "gmg_kernels.h"

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

FftQ1::~FftQ1() {
  if (fwd_ok) (void)hipfftDestroy(fft_handle(fwd));
  if (inv_ok) (void)hipfftDestroy(fft_handle(inv));
  if (spec) (void)hipFree(spec);
}

hipError_t fft_q1_prepare(FftQ1* f, int N) {
  if (f->N == N && f->fwd_ok && f->inv_ok && f->spec) return hipSuccess;
  if (N < 2) return hipErrorInvalidValue;
  const size_t bytes = sizeof(hipfftDoubleComplex) * static_cast<size_t>(N) * N * (N / 2 + 1);
  hipError_t e = hipMalloc(&f->spec, bytes);
  if (e != hipSuccess) {
    f->spec = nullptr;
    return e;
  }
  hipfftHandle h = nullptr;
  if (hipfftPlan3d(&h, N, N, N, HIPFFT_D2Z) != HIPFFT_SUCCESS) return hipErrorUnknown;
  f->fwd = h;
  f->fwd_ok = true;
  if (hipfftPlan3d(&h, N, N, N, HIPFFT_Z2D) != HIPFFT_SUCCESS) return hipErrorUnknown;
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

FftQ2::~FftQ2() {
  if (fwd_ok) (void)hipfftDestroy(fft_handle(fwd));
  if (inv_ok) (void)hipfftDestroy(fft_handle(inv));
  if (spec) (void)hipFree(spec);
  if (cls) (void)hipFree(cls);
  if (axis) (void)hipFree(axis);
}

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
    const double qa = ma * md - (mbr * mbr + mbi * mbi);
    const double qb = -(ka * md + kd * ma) + 2.0 * (kbr * mbr + kbi * mbi);
    const double qc = ka * kd - (kbr * kbr + kbi * kbi);
    const double disc = std::sqrt(std::max(0.0, qb * qb - 4.0 * qa * qc));
    Axis2& A = (*out)[k];
    A.lam[0] = (-qb - disc) / (2.0 * qa);
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

hipError_t fft_q2_prepare(FftQ2* f, int n) {
  if (f->n == n && f->fwd_ok && f->inv_ok && f->spec) return hipSuccess;
  if (n < 2 || (n & 1)) return hipErrorInvalidValue;
  const size_t n3 = static_cast<size_t>(n) * n * n;
  const size_t m = static_cast<size_t>(n) * n * (n / 2 + 1);
  if (hipMalloc(&f->spec, sizeof(hipfftDoubleComplex) * 8 * m) != hipSuccess) return hipErrorOutOfMemory;
  if (hipMalloc(&f->cls, sizeof(double) * 8 * n3) != hipSuccess) return hipErrorOutOfMemory;
  std::vector<Axis2> tab;
  q2_axis_tables(n, &tab);
  if (hipMalloc(&f->axis, sizeof(Axis2) * n) != hipSuccess) return hipErrorOutOfMemory;
  if (hipMemcpy(f->axis, tab.data(), sizeof(Axis2) * n, hipMemcpyHostToDevice) != hipSuccess) return hipErrorUnknown;
  int dims[3] = {n, n, n};
  hipfftHandle h = nullptr;
  if (hipfftPlanMany(&h, 3, dims, nullptr, 1, static_cast<int>(n3), nullptr, 1, static_cast<int>(m), HIPFFT_D2Z, 8) !=
      HIPFFT_SUCCESS)
    return hipErrorUnknown;
  f->fwd = h;
  f->fwd_ok = true;
  if (hipfftPlanMany(&h, 3, dims, nullptr, 1, static_cast<int>(m), nullptr, 1, static_cast<int>(n3), HIPFFT_Z2D, 8) !=
      HIPFFT_SUCCESS)
    return hipErrorUnknown;
  f->inv = h;
  f->inv_ok = true;
  f->n = n;
  return hipSuccess;
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
