// Intergrid transfers between nested uniform periodic meshes (Section 2.3.4,
// eqs. 2.1-2.2).  P(i, j) = phi_j^{coarse}(p_i): on uniform meshes
// P = P1 (x) P1 (x) P1, applied as three one-axis passes; R = P^T.
//
// Each pass is done element by element along its axis, with the element's
// classes compile-time:
//   prolongation: a thread takes one coarse element (q+1 coarse nodes, the
//     last shared with the next element) and writes its 2q fine nodes;
//   restriction: a thread takes one coarse element and gathers, for each of
//     its q coarse nodes, the fine nodes of the two children of that element
//     (and, for the vertex, of the element on its left): 4q+1 fine values.
// The fastest thread index always runs along x, so every access is coalesced
// whatever the pass axis.  All indices are 32-bit (N <= 2048).
#include "gmg_kernels.h"

namespace gmg {
namespace {

// K consecutive values moved as one aligned vector access (x passes: the nodes
// of one element column are contiguous and aligned to their count).
template <typename T, int K>
struct alignas(sizeof(T) * K) VecK {
  T v[K];
};

template <typename T, int Q, int AXIS, bool ACC>
__global__ void __launch_bounds__(256) k_prolong_axis(const T* __restrict__ in, T* __restrict__ out,
                                                       const TransferTab tab, const int X, const int Y,
                                                       const int Nc) {
  // output extents: X (x), Y (y); the axis extent is 2 Nc (fine), input's is Nc
  const int a0 = blockIdx.x * blockDim.x + threadIdx.x;
  const int a1 = blockIdx.y;
  const int a2 = blockIdx.z;
  const int ncm = Nc - 1;
  int E, i, j, k;
  if (AXIS == 0) {
    E = a0;
    j = a1;
    k = a2;
    if (E >= Nc / Q) return;
    i = 0;
  } else if (AXIS == 1) {
    i = a0;
    E = a1;
    k = a2;
    if (i >= X) return;
    j = 0;
  } else {
    i = a0;
    j = a1;
    E = a2;
    if (i >= X) return;
    k = 0;
  }
  // input: same extents as the output except Nc along the axis
  const int ix = AXIS == 0 ? Nc : X;
  const int iy = AXIS == 1 ? Nc : Y;
  T c[Q + 1];
  if constexpr (AXIS == 0) {
    // coarse nodes QE .. QE+Q-1 as one vector, the shared vertex QE+Q on its own
    const T* row = in + (static_cast<size_t>(k) * iy + j) * ix;
    const VecK<T, Q> cv = *reinterpret_cast<const VecK<T, Q>*>(row + Q * E);
#pragma unroll
    for (int a = 0; a < Q; ++a) c[a] = cv.v[a];
    c[Q] = row[(Q * E + Q) & ncm];
  } else {
#pragma unroll
    for (int a = 0; a <= Q; ++a) {
      const int ca = (Q * E + a) & ncm;
      int ii = i, jj = j, kk = k;
      if (AXIS == 1) jj = ca;
      else kk = ca;
      c[a] = in[(static_cast<size_t>(kk) * iy + jj) * ix + ii];
    }
  }
  if constexpr (AXIS == 0) {
    // the element's 2q fine nodes as one vector
    T* orow = out + (static_cast<size_t>(k) * Y + j) * (2 * Nc);
    VecK<T, 2 * Q> fv;
    if (ACC) fv = *reinterpret_cast<const VecK<T, 2 * Q>*>(orow + 2 * Q * E);
#pragma unroll
    for (int b = 0; b < 2 * Q; ++b) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a <= Q; ++a) s = fma(tab.p[b][a], static_cast<double>(c[a]), s);
      fv.v[b] = ACC ? static_cast<T>(static_cast<double>(fv.v[b]) + s) : static_cast<T>(s);
    }
    *reinterpret_cast<VecK<T, 2 * Q>*>(orow + 2 * Q * E) = fv;
  } else {
#pragma unroll
    for (int b = 0; b < 2 * Q; ++b) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a <= Q; ++a) s = fma(tab.p[b][a], static_cast<double>(c[a]), s);
      const int f = 2 * Q * E + b;
      int ii = i, jj = j, kk = k;
      if (AXIS == 1) jj = f;
      else kk = f;
      const int oy = AXIS == 1 ? 2 * Nc : Y;
      const size_t o = (static_cast<size_t>(kk) * oy + jj) * X + ii;
      if (ACC) out[o] = static_cast<T>(static_cast<double>(out[o]) + s);
      else out[o] = static_cast<T>(s);
    }
  }
}

template <typename T, int Q, int AXIS>
__global__ void __launch_bounds__(256) k_restrict_axis(const T* __restrict__ in, T* __restrict__ out,
                                                        const TransferTab tab, const int X, const int Y,
                                                        const int Nc) {
  const int Nf = 2 * Nc;
  const int nfm = Nf - 1;
  const int a0 = blockIdx.x * blockDim.x + threadIdx.x;
  const int a1 = blockIdx.y;
  const int a2 = blockIdx.z;
  int E, i, j, k;
  if (AXIS == 0) {
    E = a0;
    j = a1;
    k = a2;
    if (E >= Nc / Q) return;
    i = 0;
  } else if (AXIS == 1) {
    i = a0;
    E = a1;
    k = a2;
    if (i >= X) return;
    j = 0;
  } else {
    i = a0;
    j = a1;
    E = a2;
    if (i >= X) return;
    k = 0;
  }
  const int ix = AXIS == 0 ? Nf : X;
  const int iy = AXIS == 1 ? Nf : Y;
  T f[4 * Q + 1];
  if constexpr (AXIS == 0) {
    // fine nodes 2qE-2q .. 2qE+2q: two aligned vectors of 2q and the far vertex
    const T* row = in + (static_cast<size_t>(k) * iy + j) * ix;
    const VecK<T, 2 * Q> lv = *reinterpret_cast<const VecK<T, 2 * Q>*>(row + ((2 * Q * E - 2 * Q + Nf) & nfm));
    const VecK<T, 2 * Q> rv = *reinterpret_cast<const VecK<T, 2 * Q>*>(row + 2 * Q * E);
#pragma unroll
    for (int t = 0; t < 2 * Q; ++t) {
      f[t] = lv.v[t];
      f[2 * Q + t] = rv.v[t];
    }
    f[4 * Q] = row[(2 * Q * E + 2 * Q) & nfm];
  } else {
#pragma unroll
    for (int t = 0; t <= 4 * Q; ++t) {
      const int fa = (2 * Q * E - 2 * Q + t + Nf) & nfm;
      int ii = i, jj = j, kk = k;
      if (AXIS == 1) jj = fa;
      else kk = fa;
      f[t] = in[(static_cast<size_t>(kk) * iy + jj) * ix + ii];
    }
  }
  const int ox = AXIS == 0 ? Nc : X;
  const int oy = AXIS == 1 ? Nc : Y;
  VecK<T, Q> cv;
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    double s = 0.0;
#pragma unroll
    for (int t = 0; t <= 4 * Q; ++t) {
      if (a > 0 && t < 2 * Q) continue;  // only the vertex reaches into the left element
      s = fma(tab.r[a][t], static_cast<double>(f[t]), s);
    }
    cv.v[a] = static_cast<T>(s);
    if constexpr (AXIS != 0) {
      const int cidx = Q * E + a;
      int ii = i, jj = j, kk = k;
      if (AXIS == 1) jj = cidx;
      else kk = cidx;
      out[(static_cast<size_t>(kk) * oy + jj) * ox + ii] = cv.v[a];
    }
  }
  if constexpr (AXIS == 0)  // the element's q coarse nodes as one vector
    *reinterpret_cast<VecK<T, Q>*>(out + (static_cast<size_t>(k) * oy + j) * ox + Q * E) = cv;
}

constexpr int kTB = 128;

template <typename T, int Q>
hipError_t prolong3(const TransferTab& tab, const T* ec, T* t1, T* t2, T* uf, int Nc, hipStream_t s) {
  const int Nf = 2 * Nc;
  const int ne = Nc / Q;
  // x: (Nc, Nc, Nc) -> (Nf, Nc, Nc)
  hipLaunchKernelGGL((k_prolong_axis<T, Q, 0, false>), dim3((ne + kTB - 1) / kTB, Nc, Nc), dim3(kTB), 0, s, ec, t1,
                     tab, Nf, Nc, Nc);
  // y: (Nf, Nc, Nc) -> (Nf, Nf, Nc)
  hipLaunchKernelGGL((k_prolong_axis<T, Q, 1, false>), dim3((Nf + kTB - 1) / kTB, ne, Nc), dim3(kTB), 0, s, t1, t2,
                     tab, Nf, Nf, Nc);
  // z: (Nf, Nf, Nc) -> (Nf, Nf, Nf), added into uf
  hipLaunchKernelGGL((k_prolong_axis<T, Q, 2, true>), dim3((Nf + kTB - 1) / kTB, Nf, ne), dim3(kTB), 0, s, t2, uf,
                     tab, Nf, Nf, Nc);
  return hipGetLastError();
}

template <typename T, int Q>
hipError_t restrict3(const TransferTab& tab, const T* rf, T* t1, T* t2, T* rc, int Nc, hipStream_t s) {
  const int Nf = 2 * Nc;
  const int ne = Nc / Q;
  // x: (Nf, Nf, Nf) -> (Nc, Nf, Nf)
  hipLaunchKernelGGL((k_restrict_axis<T, Q, 0>), dim3((ne + kTB - 1) / kTB, Nf, Nf), dim3(kTB), 0, s, rf, t1, tab,
                     Nc, Nf, Nc);
  // y: (Nc, Nf, Nf) -> (Nc, Nc, Nf)
  hipLaunchKernelGGL((k_restrict_axis<T, Q, 1>), dim3((Nc + kTB - 1) / kTB, ne, Nf), dim3(kTB), 0, s, t1, t2, tab,
                     Nc, Nc, Nc);
  // z: (Nc, Nc, Nf) -> (Nc, Nc, Nc)
  hipLaunchKernelGGL((k_restrict_axis<T, Q, 2>), dim3((Nc + kTB - 1) / kTB, Nc, ne), dim3(kTB), 0, s, t2, rc, tab,
                     Nc, Nc, Nc);
  return hipGetLastError();
}

template <typename T>
hipError_t prolong_q(int q, const TransferTab& tab, const T* ec, T* t1, T* t2, T* uf, int Nc, hipStream_t s) {
  switch (q) {
    case 1: return prolong3<T, 1>(tab, ec, t1, t2, uf, Nc, s);
    case 2: return prolong3<T, 2>(tab, ec, t1, t2, uf, Nc, s);
    case 4: return prolong3<T, 4>(tab, ec, t1, t2, uf, Nc, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t restrict_q(int q, const TransferTab& tab, const T* rf, T* t1, T* t2, T* rc, int Nc, hipStream_t s) {
  switch (q) {
    case 1: return restrict3<T, 1>(tab, rf, t1, t2, rc, Nc, s);
    case 2: return restrict3<T, 2>(tab, rf, t1, t2, rc, Nc, s);
    case 4: return restrict3<T, 4>(tab, rf, t1, t2, rc, Nc, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_prolong(const TransferTab& tab, bool fp32, const void* ec, void* t1, void* t2, void* uf, int Nc,
                          hipStream_t s) {
  if (Nc < tab.q || (Nc & (Nc - 1)) != 0 || Nc > 1024) return hipErrorInvalidValue;
  if (fp32)
    return prolong_q<float>(tab.q, tab, static_cast<const float*>(ec), static_cast<float*>(t1),
                            static_cast<float*>(t2), static_cast<float*>(uf), Nc, s);
  return prolong_q<double>(tab.q, tab, static_cast<const double*>(ec), static_cast<double*>(t1),
                           static_cast<double*>(t2), static_cast<double*>(uf), Nc, s);
}

hipError_t launch_restrict(const TransferTab& tab, bool fp32, const void* rf, void* t1, void* t2, void* rc, int Nc,
                           hipStream_t s) {
  if (Nc < tab.q || (Nc & (Nc - 1)) != 0 || Nc > 1024) return hipErrorInvalidValue;
  if (fp32)
    return restrict_q<float>(tab.q, tab, static_cast<const float*>(rf), static_cast<float*>(t1),
                             static_cast<float*>(t2), static_cast<float*>(rc), Nc, s);
  return restrict_q<double>(tab.q, tab, static_cast<const double*>(rf), static_cast<double*>(t1),
                            static_cast<double*>(t2), static_cast<double*>(rc), Nc, s);
}

}  // namespace gmg
