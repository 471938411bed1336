// Operator apply, transfers and vector scalings on octree levels (gfx950).
//
// The octree stiffness is A = C^T blockdiag(h_e K) C (Section 2.3: element
// traversal applying the local stiffness; hanging nodes, Section 4): C maps
// the DoF vector to the (q+1)^3 nodal values of every leaf, each row one DoF
// with weight 1 or, for a hanging node, the few DoFs it is interpolated from.
// The apply is two gathers, with no atomics, so FP32 and FP64 results do not
// depend on scheduling:
//
//   k_oct_elem  one thread per element node: x_e[a] = C_(e,a) x (through LDS),
//               then y_e[a] = s_e sum_b K[a][b] x_e[b] (s_e = h or h^3 for the
//               mass); the K rows stay in LDS for the whole block
//   k_oct_dof   one thread per DoF: (A x)_k = sum over the rows of C^T of
//               w y_e[a], fused with the same epilogues as the uniform kernels
//               (apply, residual, Chebyshev step with the D^-1 vector)
//
// Transfers are CSR products with P (prolongation, fine rows) and with its
// transpose stored explicitly (restriction, coarse rows), again without atomics.
#include <algorithm>

#include "gmg_kernels.h"

namespace gmg {
namespace {

constexpr int kB = 256;

template <typename T, int M>
__global__ void __launch_bounds__(kB) k_oct_elem(const int64_t E, const uint8_t* __restrict__ lev, const int mass,
                                                 const int* __restrict__ cptr, const int* __restrict__ ccol,
                                                 const T* __restrict__ cval, const T* __restrict__ x,
                                                 const T* __restrict__ kmat, T* __restrict__ ye) {
  constexpr int EPB = kB / M;  // elements per block
  __shared__ T K[M * M];
  __shared__ T xe[EPB][M];
  for (int i = threadIdx.x; i < M * M; i += kB) K[i] = kmat[i];
  const int el = threadIdx.x / M;
  const int a = threadIdx.x - el * M;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * EPB + el;
  const bool live = el < EPB && e < E;
  if (live) {
    const int64_t r = e * M + a;
    T s = T(0);
    for (int j = cptr[r]; j < cptr[r + 1]; ++j) s = fma(cval[j], x[ccol[j]], s);
    xe[el][a] = s;
  }
  __syncthreads();
  if (live) {
    T s = T(0);
#pragma unroll 9
    for (int b = 0; b < M; ++b) s = fma(K[a * M + b], xe[el][b], s);
    const int l = lev[e];
    const T h = T(1) / static_cast<T>(1 << l);
    ye[e * M + a] = (mass ? h * h * h : h) * s;
  }
}

// Sum over one CSR row with LPR lanes per row: lane i takes entries i, i + LPR, ...,
// then a fixed butterfly of shuffles adds the lanes (the same order on every run).
// Every lane of the wave takes part in the shuffles; rows past the end add zeros.
template <typename T, int LPR, typename F>
__device__ __forceinline__ T row_sum(const int* __restrict__ ptr, int64_t row, bool live, int sub, F term) {
  T s = T(0);
  if (live)
    for (int j = ptr[row] + sub; j < ptr[row + 1]; j += LPR) s += term(j);
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

template <typename T, int EPI, int LPR>
__global__ void __launch_bounds__(kB) k_oct_dof(const int64_t n, const int* __restrict__ tptr,
                                                const int* __restrict__ trow, const T* __restrict__ tval,
                                                const T* __restrict__ ye, const T* __restrict__ x,
                                                const T* __restrict__ b, const T* xp, const T* __restrict__ dinv,
                                                const T c1, const T c2, T* out) {
  const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t k = t / LPR;
  const int sub = static_cast<int>(t % LPR);
  const bool live = k < n;
  const T ax = row_sum<T, LPR>(tptr, k, live, sub, [&](int j) { return tval[j] * ye[trow[j]]; });
  if (!live || sub != 0) return;
  if constexpr (EPI == static_cast<int>(Epi::Apply)) {
    out[k] = ax;
  } else if constexpr (EPI == static_cast<int>(Epi::Residual)) {
    out[k] = b[k] - ax;
  } else {
    const T xv = x[k];
    const T pv = (c1 != T(0)) ? (xp ? xp[k] : T(0)) : xv;
    out[k] = xv + c1 * (xv - pv) + c2 * dinv[k] * (b[k] - ax);
  }
}

// y (+)= A x for a CSR matrix, LPR lanes per row
template <typename T, bool ACC, int LPR>
__global__ void __launch_bounds__(kB) k_csr(const int64_t rows, const int* __restrict__ ptr,
                                            const int* __restrict__ col, const T* __restrict__ val,
                                            const T* __restrict__ x, T* __restrict__ y) {
  const int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t i = t / LPR;
  const int sub = static_cast<int>(t % LPR);
  const bool live = i < rows;
  const T s = row_sum<T, LPR>(ptr, i, live, sub, [&](int j) { return val[j] * x[col[j]]; });
  if (!live || sub != 0) return;
  if (ACC) y[i] += s;
  else y[i] = s;
}

// out = c d (.* in)   (in may be null: out = c d; d may be null: d = 1)
template <typename T>
__global__ void __launch_bounds__(kB) k_vscale(const int64_t n, const double* d, const double c, const T* in,
                                               T* out) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double f = d ? c * d[i] : c;
    out[i] = static_cast<T>(in ? f * static_cast<double>(in[i]) : f);
  }
}

// blocks for one thread per item (lanes = 1) or `lanes` threads per row; no grid-stride loop
inline int grid_rows(int64_t rows, int lanes) { return static_cast<int>((rows * lanes + kB - 1) / kB); }
inline int grid(int64_t n) { return static_cast<int>(std::min<int64_t>((n + kB - 1) / kB, 8192)); }

constexpr int kDofLanes = 4;       // rows of C^T: the element nodes of one DoF (8 to ~30)
constexpr int kProlongLanes = 4;   // rows of P: up to (q+1)^3 coarse DoFs
constexpr int kRestrictLanes = 16; // rows of P^T: up to (2q+1)^3 fine DoFs

template <typename T, int M>
hipError_t elem(const OctLevelDev& L, bool mass, const T* x, const T* cval, const T* kmat, T* ye, hipStream_t s) {
  constexpr int EPB = kB / M;
  const int blocks = static_cast<int>((L.E + EPB - 1) / EPB);
  hipLaunchKernelGGL((k_oct_elem<T, M>), dim3(blocks), dim3(kB), 0, s, L.E, L.lev, mass ? 1 : 0, L.cptr, L.ccol,
                     cval, x, kmat, ye);
  return hipGetLastError();
}

template <typename T>
hipError_t apply_t(const OctLevelDev& L, bool mass, const OctApply& a, hipStream_t s) {
  if (a.epi == Epi::ChebZero) return hipErrorInvalidValue;
  const T* x = static_cast<const T*>(a.x);
  T* ye = static_cast<T*>(a.ye);
  const bool f32 = sizeof(T) == 4;
  const T* cval = static_cast<const T*>(f32 ? static_cast<const void*>(L.cval32) : L.cval64);
  const T* tval = static_cast<const T*>(f32 ? static_cast<const void*>(L.tval32) : L.tval64);
  const T* kmat = static_cast<const T*>(f32 ? static_cast<const void*>(mass ? L.mref32 : L.kref32)
                                            : static_cast<const void*>(mass ? L.mref64 : L.kref64));
  const T* dinv = static_cast<const T*>(f32 ? static_cast<const void*>(L.dinv32) : L.dinv64);
  hipError_t e = (L.m == 27) ? elem<T, 27>(L, mass, x, cval, kmat, ye, s) : elem<T, 8>(L, mass, x, cval, kmat, ye, s);
  if (e != hipSuccess) return e;
  const T* b = static_cast<const T*>(a.b);
  const T* xp = static_cast<const T*>(a.xp);
  T* out = static_cast<T*>(a.out);
  const T c1 = static_cast<T>(a.c1), c2 = static_cast<T>(a.c2);
  const dim3 g(grid_rows(L.n, kDofLanes));
  switch (a.epi) {
    case Epi::Apply:
      hipLaunchKernelGGL((k_oct_dof<T, 0, kDofLanes>), g, dim3(kB), 0, s, L.n, L.tptr, L.trow, tval, ye, x, b, xp,
                         dinv, c1, c2, out);
      break;
    case Epi::Residual:
      hipLaunchKernelGGL((k_oct_dof<T, 1, kDofLanes>), g, dim3(kB), 0, s, L.n, L.tptr, L.trow, tval, ye, x, b, xp,
                         dinv, c1, c2, out);
      break;
    case Epi::Cheb:
      hipLaunchKernelGGL((k_oct_dof<T, 2, kDofLanes>), g, dim3(kB), 0, s, L.n, L.tptr, L.trow, tval, ye, x, b, xp,
                         dinv, c1, c2, out);
      break;
    default:
      return hipErrorInvalidValue;  // the zero-guess step and the reducing epilogues: uniform levels only
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_oct_apply(const OctLevelDev& L, bool fp32, bool mass, const OctApply& a, hipStream_t s) {
  return fp32 ? apply_t<float>(L, mass, a, s) : apply_t<double>(L, mass, a, s);
}

hipError_t launch_oct_prolong(const OctLevelDev& F, bool fp32, const void* ec, void* uf, hipStream_t s) {
  const dim3 g(grid_rows(F.n, kProlongLanes));
  if (fp32)
    hipLaunchKernelGGL((k_csr<float, true, kProlongLanes>), g, dim3(kB), 0, s, F.n, F.pptr, F.pcol, F.pval32,
                       static_cast<const float*>(ec), static_cast<float*>(uf));
  else
    hipLaunchKernelGGL((k_csr<double, true, kProlongLanes>), g, dim3(kB), 0, s, F.n, F.pptr, F.pcol, F.pval64,
                       static_cast<const double*>(ec), static_cast<double*>(uf));
  return hipGetLastError();
}

hipError_t launch_oct_restrict(const OctLevelDev& F, int64_t nc, bool fp32, const void* rf, void* rc, hipStream_t s) {
  const dim3 g(grid_rows(nc, kRestrictLanes));
  if (fp32)
    hipLaunchKernelGGL((k_csr<float, false, kRestrictLanes>), g, dim3(kB), 0, s, nc, F.rptr, F.rcol, F.rval32,
                       static_cast<const float*>(rf), static_cast<float*>(rc));
  else
    hipLaunchKernelGGL((k_csr<double, false, kRestrictLanes>), g, dim3(kB), 0, s, nc, F.rptr, F.rcol, F.rval64,
                       static_cast<const double*>(rf), static_cast<double*>(rc));
  return hipGetLastError();
}

hipError_t launch_vec_scale(bool fp32, int64_t n, const double* d, double c, const void* in, void* out,
                            hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_vscale<float>, dim3(grid(n)), dim3(kB), 0, s, n, d, c, static_cast<const float*>(in),
                       static_cast<float*>(out));
  else
    hipLaunchKernelGGL(k_vscale<double>, dim3(grid(n)), dim3(kB), 0, s, n, d, c, static_cast<const double*>(in),
                       static_cast<double*>(out));
  return hipGetLastError();
}

}  // namespace gmg
