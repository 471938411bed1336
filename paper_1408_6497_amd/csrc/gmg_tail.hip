// The V-cycle's work on the level of 16^3 nodes whose next coarser level is the
// coarsest (8^3 nodes, solved directly), in one workgroup with the whole level
// in LDS (Algorithm 2.1 on that level; smoother, Section 2.3.3; transfers,
// eq. 2.2 and Section 2.3.4).
//
// On a level this small every separate kernel costs its launch and ramp (about
// 5 us on gfx950) for a few microseconds of work, and the level takes about 20
// of them per cycle.  Here two launches do the same steps:
//
//   k_tail_down  u = 0, the pre-smoothing steps, r = b - A u, b_c = P^T r
//   (the coarsest solve runs in between, as its own launch)
//   k_tail_up    u += P e_c, the post-smoothing steps
//
// 1024 threads, 4 nodes each (node t + 1024 m); the iterate, the right side and
// the previous iterate of a thread's nodes stay in registers, and the level
// vectors pass through four LDS arrays of 16^3 values.  The operator is applied
// by sum factorization in three banded passes (z, then y, then x) over the
// assembled periodic 1D rows, the smoother steps are the Chebyshev (or Jacobi)
// recurrence x' = x + c1 (x - x_prev) + c2 D^-1 (b - A x) with the host's
// coefficients, and the transfers use the same one-axis weights, summation
// order and FP64 accumulation as the transfer kernels.
#include <algorithm>

#include "gmg_kernels.h"

namespace gmg {
namespace {

constexpr int kTN = 16;               // nodes a side of the level
constexpr int kTV = kTN * kTN * kTN;  // nodes of the level
constexpr int kTT = 1024;             // threads of the workgroup
constexpr int kPer = kTV / kTT;       // nodes per thread
constexpr int kNc = kTN / 2;          // nodes a side of the coarsest level

template <typename T, int Q>
struct TailTab {
  T kr[Q][2 * Q + 1];   // assembled 1D stiffness rows by node class, offsets -q..q (x, y)
  T mr[Q][2 * Q + 1];   // assembled 1D mass rows
  T zkr[Q][2 * Q + 1];  // the same for the z direction
  T zmr[Q][2 * Q + 1];
  T dinv[Q * Q * Q];    // D^-1 by node class
  double p[2 * Q][Q + 1];
  double r[Q][4 * Q + 1];
  T c1[kTailMaxSteps];  // smoother steps: npre pre-smoothing steps, then npost post-smoothing steps
  T c2[kTailMaxSteps];
  int npre, npost;
};

__device__ __forceinline__ int node(int m) { return static_cast<int>(threadIdx.x) + kTT * m; }

template <int Q>
__device__ __forceinline__ int node_class(int idx) {
  const int i = idx & 15, j = (idx >> 4) & 15, k = idx >> 8;
  return (i % Q) + Q * ((j % Q) + Q * (k % Q));
}

// ax = (A x) at this thread's nodes, x in X (all nodes).  X, A1, A2 and A3 are
// clobbered; on return every thread is past its last read of them.
//
// A thread's nodes t + 1024 m share i = t mod 16, j = (t / 16) mod 16 and
// k mod q (1024 is 4 planes and q divides 4), so they share one node class: each
// pass loads the thread's two 1D rows into registers once and runs all 2q+1 taps
// (the weights outside a row's band are zero).  FP32 with q <= 2 keeps a
// thread's 4 nodes in flight at once; the others take them one at a time
// (unrolled, they would exceed the 128 registers a 1024-thread block allows).
template <typename T, int Q>
__device__ void tail_apply(const TailTab<T, Q>& tb, T* X, T* A1, T* A2, T* A3, T (&ax)[kPer]) {
  constexpr int kU = (sizeof(T) == 4 && Q <= 2) ? kPer : 1;  // nodes in flight per thread
  const int t = static_cast<int>(threadIdx.x);
  const int i = t & 15, j = (t >> 4) & 15, k0 = t >> 8;
  T ra[2 * Q + 1], rb[2 * Q + 1];
  // z: A1 = Mz x, A2 = Kz x
  {
    const int cz = k0 % Q;
#pragma unroll
    for (int o = 0; o <= 2 * Q; ++o) {
      ra[o] = tb.zmr[cz][o];
      rb[o] = tb.zkr[cz][o];
    }
  }
#pragma unroll kU
  for (int m = 0; m < kPer; ++m) {
    const int k = k0 + 4 * m;
    T tm = T(0), tk = T(0);
#pragma unroll
    for (int o = -Q; o <= Q; ++o) {
      const T v = X[i + kTN * (j + kTN * ((k + o) & 15))];
      tm = fma(ra[o + Q], v, tm);
      tk = fma(rb[o + Q], v, tk);
    }
    const int idx = i + kTN * (j + kTN * k);
    A1[idx] = tm;
    A2[idx] = tk;
  }
  __syncthreads();
  // y: X = My A1, A3 = Ky A1 + My A2 (x itself is not read again)
  {
    const int cy = j % Q;
#pragma unroll
    for (int o = 0; o <= 2 * Q; ++o) {
      ra[o] = tb.mr[cy][o];
      rb[o] = tb.kr[cy][o];
    }
  }
#pragma unroll kU
  for (int m = 0; m < kPer; ++m) {
    const int k = k0 + 4 * m;
    T u1 = T(0), u2 = T(0);
#pragma unroll
    for (int o = -Q; o <= Q; ++o) {
      const int at = i + kTN * (((j + o) & 15) + kTN * k);
      const T a1 = A1[at], a2 = A2[at];
      u1 = fma(ra[o + Q], a1, u1);
      u2 = fma(rb[o + Q], a1, fma(ra[o + Q], a2, u2));
    }
    const int idx = i + kTN * (j + kTN * k);
    X[idx] = u1;
    A3[idx] = u2;
  }
  __syncthreads();
  // x: A x = Kx X + Mx A3
  {
    const int cx = i % Q;
#pragma unroll
    for (int o = 0; o <= 2 * Q; ++o) {
      ra[o] = tb.mr[cx][o];
      rb[o] = tb.kr[cx][o];
    }
  }
#pragma unroll kU
  for (int m = 0; m < kPer; ++m) {
    const int k = k0 + 4 * m;
    T s = T(0);
#pragma unroll
    for (int o = -Q; o <= Q; ++o) {
      const int at = ((i + o) & 15) + kTN * (j + kTN * k);
      s = fma(rb[o + Q], X[at], fma(ra[o + Q], A3[at], s));
    }
    ax[m] = s;
  }
  __syncthreads();
}

// Smoother steps s0 .. s1-1 on x (registers, mirrored in X); x_prev starts as xp.
// zero: x = 0 on entry, so the first step needs no operator apply.
template <typename T, int Q>
__device__ void tail_smooth(const TailTab<T, Q>& tb, int s0, int s1, bool zero, T (&x)[kPer], T (&xp)[kPer],
                            const T (&b)[kPer], T* X, T* A1, T* A2, T* A3) {
  for (int st = s0; st < s1; ++st) {
    T ax[kPer];
    if (zero && st == s0) {
#pragma unroll
      for (int m = 0; m < kPer; ++m) ax[m] = T(0);
    } else {
      tail_apply<T, Q>(tb, X, A1, A2, A3, ax);
    }
    const T c1 = tb.c1[st], c2 = tb.c2[st];
    const T dv = tb.dinv[node_class<Q>(node(0))];  // the same class for all of the thread's nodes
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
      const int idx = node(m);
      const T xn = x[m] + c1 * (x[m] - xp[m]) + c2 * dv * (b[m] - ax[m]);
      xp[m] = x[m];
      x[m] = xn;
      X[idx] = xn;
    }
    __syncthreads();
  }
}

template <typename T, int Q>
__global__ void __launch_bounds__(kTT) k_tail_down(const TailTab<T, Q> tb, const T* __restrict__ bg,
                                                   T* __restrict__ ug, T* __restrict__ bc) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* X = reinterpret_cast<T*>(smem_raw);
  T* A1 = X + kTV;
  T* A2 = A1 + kTV;
  T* A3 = A2 + kTV;
  T x[kPer], xp[kPer], b[kPer];
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    b[m] = bg[node(m)];
    x[m] = T(0);
    xp[m] = T(0);
  }
  tail_smooth<T, Q>(tb, 0, tb.npre, true, x, xp, b, X, A1, A2, A3);
  if (tb.npre == 0) {
#pragma unroll
    for (int m = 0; m < kPer; ++m) X[node(m)] = T(0);
    __syncthreads();
  }
  // r = b - A u into A1, u to global memory
  T ax[kPer];
  tail_apply<T, Q>(tb, X, A1, A2, A3, ax);
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    const int idx = node(m);
    ug[idx] = x[m];
    A1[idx] = b[m] - ax[m];
  }
  __syncthreads();
  // b_c = P^T r, one axis at a time: x (16,16,16) -> (8,16,16) in A2
  for (int o = threadIdx.x; o < kNc * kTN * kTN; o += kTT) {
    const int ci = o % kNc, j = (o / kNc) % kTN, k = o / (kNc * kTN);
    const int E = ci / Q, a = ci % Q;
    double s = 0.0;
#pragma unroll
    for (int t = 0; t <= 4 * Q; ++t) {
      if (a > 0 && t < 2 * Q) continue;  // only the vertex reaches into the left element
      s = fma(tb.r[a][t], static_cast<double>(A1[((2 * Q * E - 2 * Q + t) & 15) + kTN * (j + kTN * k)]), s);
    }
    A2[o] = static_cast<T>(s);
  }
  __syncthreads();
  // y: (8,16,16) -> (8,8,16) in A3
  for (int o = threadIdx.x; o < kNc * kNc * kTN; o += kTT) {
    const int ci = o % kNc, cj = (o / kNc) % kNc, k = o / (kNc * kNc);
    const int E = cj / Q, a = cj % Q;
    double s = 0.0;
#pragma unroll
    for (int t = 0; t <= 4 * Q; ++t) {
      if (a > 0 && t < 2 * Q) continue;
      s = fma(tb.r[a][t], static_cast<double>(A2[ci + kNc * (((2 * Q * E - 2 * Q + t) & 15) + kTN * k)]), s);
    }
    A3[o] = static_cast<T>(s);
  }
  __syncthreads();
  // z: (8,8,16) -> (8,8,8) to the coarsest level's right side
  for (int o = threadIdx.x; o < kNc * kNc * kNc; o += kTT) {
    const int ci = o % kNc, cj = (o / kNc) % kNc, ck = o / (kNc * kNc);
    const int E = ck / Q, a = ck % Q;
    double s = 0.0;
#pragma unroll
    for (int t = 0; t <= 4 * Q; ++t) {
      if (a > 0 && t < 2 * Q) continue;
      s = fma(tb.r[a][t], static_cast<double>(A3[ci + kNc * (cj + kNc * ((2 * Q * E - 2 * Q + t) & 15))]), s);
    }
    bc[o] = static_cast<T>(s);
  }
}

template <typename T, int Q>
__global__ void __launch_bounds__(kTT) k_tail_up(const TailTab<T, Q> tb, const T* __restrict__ bg,
                                                 T* __restrict__ ug, const T* __restrict__ ec) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* X = reinterpret_cast<T*>(smem_raw);
  T* A1 = X + kTV;
  T* A2 = A1 + kTV;
  T* A3 = A2 + kTV;
  for (int o = threadIdx.x; o < kNc * kNc * kNc; o += kTT) A1[o] = ec[o];
  __syncthreads();
  // u += P e_c, one axis at a time: x (8,8,8) -> (16,8,8) in A2
  for (int o = threadIdx.x; o < kTN * kNc * kNc; o += kTT) {
    const int fi = o % kTN, cj = (o / kTN) % kNc, ck = o / (kTN * kNc);
    const int E = fi / (2 * Q), bb = fi % (2 * Q);
    double s = 0.0;
#pragma unroll
    for (int a = 0; a <= Q; ++a)
      s = fma(tb.p[bb][a], static_cast<double>(A1[((Q * E + a) & (kNc - 1)) + kNc * (cj + kNc * ck)]), s);
    A2[o] = static_cast<T>(s);
  }
  __syncthreads();
  // y: (16,8,8) -> (16,16,8) in A3
  for (int o = threadIdx.x; o < kTN * kTN * kNc; o += kTT) {
    const int fi = o % kTN, fj = (o / kTN) % kTN, ck = o / (kTN * kTN);
    const int E = fj / (2 * Q), bb = fj % (2 * Q);
    double s = 0.0;
#pragma unroll
    for (int a = 0; a <= Q; ++a)
      s = fma(tb.p[bb][a], static_cast<double>(A2[fi + kTN * (((Q * E + a) & (kNc - 1)) + kNc * ck)]), s);
    A3[o] = static_cast<T>(s);
  }
  __syncthreads();
  // z: (16,16,8) -> (16,16,16), added to u
  T x[kPer], xp[kPer], b[kPer];
  constexpr int kU = (sizeof(T) == 4 && Q <= 2) ? kPer : 1;
#pragma unroll kU
  for (int m = 0; m < kPer; ++m) {
    const int idx = node(m);
    const int i = idx & 15, j = (idx >> 4) & 15, k = idx >> 8;
    const int E = k / (2 * Q), bb = k % (2 * Q);
    double s = 0.0;
#pragma unroll
    for (int a = 0; a <= Q; ++a)
      s = fma(tb.p[bb][a], static_cast<double>(A3[i + kTN * (j + kTN * ((Q * E + a) & (kNc - 1)))]), s);
    x[m] = static_cast<T>(static_cast<double>(ug[idx]) + s);
    xp[m] = x[m];
    b[m] = bg[idx];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < kPer; ++m) X[node(m)] = x[m];
  __syncthreads();
  tail_smooth<T, Q>(tb, tb.npre, tb.npre + tb.npost, false, x, xp, b, X, A1, A2, A3);
#pragma unroll
  for (int m = 0; m < kPer; ++m) ug[node(m)] = x[m];
}

template <typename T, int Q>
TailTab<T, Q> make_tail_tab(const OpTab& op, const TransferTab& xf, const TailSteps& st) {
  TailTab<T, Q> t{};
  for (int c = 0; c < Q; ++c)
    for (int o = 0; o < 2 * Q + 1; ++o) {
      t.kr[c][o] = static_cast<T>(op.krow[c][o]);
      t.mr[c][o] = static_cast<T>(op.mrow[c][o]);
      t.zkr[c][o] = static_cast<T>(op.zkrow[c][o]);
      t.zmr[c][o] = static_cast<T>(op.zmrow[c][o]);
    }
  for (int i = 0; i < Q * Q * Q; ++i) t.dinv[i] = static_cast<T>(op.dinv[i]);
  for (int b = 0; b < 2 * Q; ++b)
    for (int a = 0; a <= Q; ++a) t.p[b][a] = xf.p[b][a];
  for (int a = 0; a < Q; ++a)
    for (int k = 0; k <= 4 * Q; ++k) t.r[a][k] = xf.r[a][k];
  for (int s = 0; s < st.npre + st.npost; ++s) {
    t.c1[s] = static_cast<T>(st.c1[s]);
    t.c2[s] = static_cast<T>(st.c2[s]);
  }
  t.npre = st.npre;
  t.npost = st.npost;
  return t;
}

template <typename T, int Q>
hipError_t tail_tq(bool up, const OpTab& op, const TransferTab& xf, const TailSteps& st, const void* b, void* u,
                   void* c, hipStream_t s) {
  const TailTab<T, Q> tb = make_tail_tab<T, Q>(op, xf, st);
  const size_t lds = 4 * static_cast<size_t>(kTV) * sizeof(T);
  const void* fn = up ? reinterpret_cast<const void*>(&k_tail_up<T, Q>) : reinterpret_cast<const void*>(&k_tail_down<T, Q>);
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  if (up)
    hipLaunchKernelGGL((k_tail_up<T, Q>), dim3(1), dim3(kTT), lds, s, tb, static_cast<const T*>(b), static_cast<T*>(u),
                       static_cast<const T*>(c));
  else
    hipLaunchKernelGGL((k_tail_down<T, Q>), dim3(1), dim3(kTT), lds, s, tb, static_cast<const T*>(b),
                       static_cast<T*>(u), static_cast<T*>(c));
  return hipGetLastError();
}

template <typename T>
hipError_t tail_t(bool up, const OpTab& op, const TransferTab& xf, const TailSteps& st, const void* b, void* u,
                  void* c, hipStream_t s) {
  switch (op.q) {
    case 1: return tail_tq<T, 1>(up, op, xf, st, b, u, c, s);
    case 2: return tail_tq<T, 2>(up, op, xf, st, b, u, c, s);
    case 4:
      if constexpr (sizeof(T) == 4) return tail_tq<T, 4>(up, op, xf, st, b, u, c, s);
      break;
  }
  return hipErrorInvalidValue;
}

}  // namespace

// FP64 q = 4 is left to the separate kernels: its up pass spills registers and
// measured no faster than the launches it replaces.
bool tail_supported(int q, bool fp32, int N, int Nc, const TailSteps& st) {
  return (q == 1 || q == 2 || (q == 4 && fp32)) && N == kTN && Nc == kNc && st.npre >= 0 && st.npost >= 0 &&
         st.npre + st.npost <= kTailMaxSteps;
}

hipError_t launch_tail_down(const OpTab& op, const TransferTab& xf, const TailSteps& st, bool fp32, const void* b,
                            void* u, void* bc, hipStream_t s) {
  if (!tail_supported(op.q, fp32, kTN, kNc, st) || xf.q != op.q) return hipErrorInvalidValue;
  return fp32 ? tail_t<float>(false, op, xf, st, b, u, bc, s) : tail_t<double>(false, op, xf, st, b, u, bc, s);
}

hipError_t launch_tail_up(const OpTab& op, const TransferTab& xf, const TailSteps& st, bool fp32, const void* b,
                          void* u, const void* ec, hipStream_t s) {
  if (!tail_supported(op.q, fp32, kTN, kNc, st) || xf.q != op.q) return hipErrorInvalidValue;
  return fp32 ? tail_t<float>(true, op, xf, st, b, u, const_cast<void*>(ec), s)
              : tail_t<double>(true, op, xf, st, b, u, const_cast<void*>(ec), s);
}

}  // namespace gmg
