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
