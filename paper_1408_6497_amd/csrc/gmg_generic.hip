// Operator, transfers and diagonal-class arithmetic of uniform periodic levels whose
// order has no specialised kernel: q = 3 and 5 .. 16 (Section 2.3.2 admits 1 <= q <= 16;
// Table 10 runs q = 4, 5, 6, 8, Table 7 q = 14 and 16).  N = q n lattice nodes per direction, n a power of two
// (n = 1 allowed: a single periodic element), so N is not a power of two in general and
// every periodic index is taken modulo N.
//
// The operator A = Kx (x) My (x) Mz + Mx (x) Ky (x) Mz + Mx (x) My (x) Kz is applied in the
// tile form, as three banded 1D passes through global memory:
//   z pass   T1 = Mz x,            T2 = Kz x
//   y pass   U1 = My T1,           V  = Ky T1 + My T2
//   x pass   y  = Kx U1 + Mx V,    with the epilogue (residual, smoother step)
// Row c of a 1D matrix (node class c = i mod q) has 2q+1 taps at offsets -q..q; every
// node is touched once per pass (14 (q+2) flops per DoF) at the cost of four temporaries.
// The mass M (x) M (x) M goes through the same passes with Kz = Ky = 0 and the x pass's
// K row set to M.  Each pass is compiled per order: a thread takes one element segment of
// a lattice line (its q nodes), loads the 2q+1 values its rows reach once and writes q
// outputs (the z and y passes always; the x pass as set by gen_x_lds and gen_x_per_element,
// else a thread per node).  Transfers P = P1 (x) P1 (x) P1 and P^T are three one-axis passes
// each, a thread per coarse element of a line (a thread per output node for an order without
// an instance).  These levels trade the fused streaming kernels of q = 1, 2, 4 for generality.
#include "gmg_kernels.h"

namespace gmg {
namespace {

constexpr int kGB = 256;
// The x pass: staged through LDS (k_gen_pass_xl) when N / q divides its block, except for the
// smoother step at q <= 5; else in the per-element register form (k_gen_pass_x) for the apply
// and the residual, and for the smoother step up to q = 7; else a thread per node
// (k_gen_pass).  Measured near 256^3 DoFs against the register and per-node forms: the LDS
// form takes the FP32 apply 21-25 % and the FP64 apply 13-29 % faster at q = 8, 14, 16 and
// FP32-cycle solves 6 % (q = 6) to 23 % (q = 16) faster; at q = 3, 5 the applies are even and
// the solves about 1 % slower with it, hence the register form's smoother step there.
inline bool gen_x_lds(int q, Epi epi) { return epi != Epi::Cheb || q >= 6; }
inline bool gen_x_per_element(int q, Epi epi) { return epi != Epi::Cheb || q <= 7; }

inline unsigned gen_grid(int64_t n) {
  int64_t g = (n + kGB - 1) / kGB;
  if (g > 1 << 30) g = 1 << 30;
  return static_cast<unsigned>(g < 1 ? 1 : g);
}

// i mod N for -N <= i < 2N (every shifted index below: a node index plus a tap offset of
// at most one element's span, and a level is at least one element wide), by two selects
// instead of an integer division per tap
__device__ __forceinline__ int wrap(int i, int N) {
  i += i < 0 ? N : 0;
  return i >= N ? i - N : i;
}

// (i, j, k) of a flat index with x fastest; every extent here has at most 1024^3 < 2^31
// nodes, so 32-bit divisions suffice
__device__ __forceinline__ void split3(int64_t idx, int X, int Y, int& i, int& j, int& k) {
  const uint32_t u = static_cast<uint32_t>(idx);
  const uint32_t jk = u / static_cast<uint32_t>(X);
  i = static_cast<int>(u - jk * static_cast<uint32_t>(X));
  k = static_cast<int>(jk / static_cast<uint32_t>(Y));
  j = static_cast<int>(jk - static_cast<uint32_t>(k) * static_cast<uint32_t>(Y));
}

// one banded pass along AXIS; T1/T2 (z), U1/V (y) or the output (x)
// rows: 6 blocks of q (2q+1): z K, z M, y K, y M, x K, x M
template <typename T, int AXIS, int EPI>
__global__ void __launch_bounds__(kGB) k_gen_pass(const T* __restrict__ in0, const T* __restrict__ in1,
                                                   const T* __restrict__ rows, const T* __restrict__ dinv, const int q,
                                                   const int N, T* __restrict__ out0, T* __restrict__ out1,
                                                   const T* __restrict__ x, const T* __restrict__ b,
                                                   const T* xp, const T c1, const T c2) {
  __shared__ T rk[kGenMaxQ * (2 * kGenMaxQ + 1)], rm[kGenMaxQ * (2 * kGenMaxQ + 1)];
  const int w = 2 * q + 1;
  const int blk = q * w;
  const T* kr = rows + (2 * AXIS) * blk;
  for (int e = threadIdx.x; e < blk; e += blockDim.x) {
    rk[e] = kr[e];
    rm[e] = kr[blk + e];
  }
  __syncthreads();
  const int64_t n3 = static_cast<int64_t>(N) * N * N;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < n3;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int i, j, k;
    split3(idx, N, N, i, j, k);
    const int a = AXIS == 2 ? i : (AXIS == 1 ? j : k);   // coordinate along the pass
    const int c = a % q;
    const T* rkc = rk + c * w;
    const T* rmc = rm + c * w;
    T s0 = T(0), s1 = T(0);
    for (int o = -q; o <= q; ++o) {
      const int aa = wrap(a + o, N);
      int64_t src;
      if (AXIS == 0) src = (static_cast<int64_t>(aa) * N + j) * N + i;
      else if (AXIS == 1) src = (static_cast<int64_t>(k) * N + aa) * N + i;
      else src = (static_cast<int64_t>(k) * N + j) * N + aa;
      const T kv = rkc[o + q], mv = rmc[o + q];
      if (AXIS == 0) {                       // T1 = M x, T2 = K x
        const T v = in0[src];
        s0 += mv * v;
        s1 += kv * v;
      } else if (AXIS == 1) {                // U1 = M T1, V = K T1 + M T2
        const T t1 = in0[src], t2 = in1[src];
        s0 += mv * t1;
        s1 += kv * t1 + mv * t2;
      } else {                               // y = K U1 + M V
        s0 += kv * in0[src] + mv * in1[src];
      }
    }
    if constexpr (AXIS < 2) {
      out0[idx] = s0;
      out1[idx] = s1;
    } else if constexpr (EPI == static_cast<int>(Epi::Apply)) {
      out0[idx] = s0;
    } else if constexpr (EPI == static_cast<int>(Epi::Residual)) {
      out0[idx] = b[idx] - s0;
    } else {  // Epi::Cheb: x + c1 (x - xp) + c2 D^-1 (b - A x); xp read as 0 when null
      const int cls = (i % q) + q * ((j % q) + q * (k % q));
      const T xv = x[idx];
      const T xpv = (xp != nullptr && c1 != T(0)) ? xp[idx] : T(0);
      out0[idx] = xv + c1 * (xv - xpv) + c2 * dinv[cls] * (b[idx] - s0);
    }
  }
}

// The z and y passes for order Q: a thread takes one element segment of a lattice line along
// the pass (its Q nodes), loads the 2Q+1 values its rows reach once (the segment, its right
// vertex and, for the vertex row, the left element) and writes its Q outputs, skipping the
// structurally zero taps; consecutive threads take consecutive x, so every load is coalesced.
// The weights are uniform (scalar loads).  AXIS 0: T1 = M x, T2 = K x; AXIS 1: U1 = M T1,
// V = K T1 + M T2.
// The z or y pass for order Q: a thread takes C (1 or 2) consecutive element segments of one
// lattice line (lanes along x, so every load and store is coalesced), loads the 2q+1-value
// window of the first and, for the next, only its q new values (the q+1 it shares with the
// previous window stay in registers), and writes q outputs per element.
template <typename T, int Q, int AXIS, int C>
__global__ void __launch_bounds__(kGB) k_gen_pass_zy(const T* __restrict__ in0, const T* __restrict__ in1,
                                                      const T* __restrict__ rows, const int N,
                                                      T* __restrict__ out0, T* __restrict__ out1) {
  static_assert(AXIS == 0 || AXIS == 1, "z and y passes");
  constexpr int W = 2 * Q + 1;
  constexpr bool kTwo = AXIS == 1;
  const T* __restrict__ kr = rows + (2 * AXIS) * (Q * W);
  const T* __restrict__ mr = kr + Q * W;
  const int nC = N / Q / C;
  const int64_t total = static_cast<int64_t>(nC) * N * N;
  const int64_t step = AXIS == 0 ? static_cast<int64_t>(N) * N : N;  // along the line
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int i, m, ch;  // x; the other coordinate across the line (y for AXIS 0, z for AXIS 1); chunk
    if constexpr (AXIS == 0) split3(t, N, N, i, m, ch);
    else split3(t, N, nC, i, ch, m);
    const int64_t base = AXIS == 0 ? static_cast<int64_t>(m) * N + i : static_cast<int64_t>(m) * N * N + i;
    const int e0 = ch * C;
    T w0[W], w1[kTwo ? W : 1];
#pragma unroll
    for (int u = 0; u < W; ++u) {
      const int64_t at = base + static_cast<int64_t>(wrap(e0 * Q - Q + u, N)) * step;
      w0[u] = in0[at];
      if constexpr (kTwo) w1[u] = in1[at];
    }
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const int e = e0 + k;
      T n0[Q], n1[kTwo ? Q : 1];
      if (k + 1 < C) {  // the next element's new values, in flight while this one computes
#pragma unroll
        for (int u = 0; u < Q; ++u) {
          const int64_t at = base + static_cast<int64_t>(wrap(e * Q + Q + 1 + u, N)) * step;
          n0[u] = in0[at];
          if constexpr (kTwo) n1[u] = in1[at];
        }
      }
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        T s0 = T(0), s1 = T(0);
#pragma unroll
        for (int o = -Q; o <= Q; ++o) {
          if (c != 0 && (o < -c || o > Q - c)) continue;  // structural zero of row c
          const T kv = kr[c * W + o + Q], mv = mr[c * W + o + Q];
          const T v0 = w0[c + o + Q];
          s0 = fma(mv, v0, s0);
          s1 = fma(kv, v0, s1);
          if constexpr (kTwo) s1 = fma(mv, w1[c + o + Q], s1);
        }
        const int64_t at = base + static_cast<int64_t>(e * Q + c) * step;
        out0[at] = s0;
        out1[at] = s1;
      }
      if (k + 1 < C) {
#pragma unroll
        for (int u = 0; u <= Q; ++u) {
          w0[u] = w0[u + Q];
          if constexpr (kTwo) w1[u] = w1[u + Q];
        }
#pragma unroll
        for (int u = 0; u < Q; ++u) {
          w0[Q + 1 + u] = n0[u];
          if constexpr (kTwo) w1[Q + 1 + u] = n1[u];
        }
      }
    }
  }
}

// The z or y pass for order Q staged through LDS: a block takes kZlLanes consecutive x lanes of
// one plane across the line (y for the z pass, z for the y pass) and ZT consecutive elements
// along it, loads the (ZT + 1) q + 1 lattice rows their windows span once (coalesced along x),
// and each thread computes one element segment of one lane from its 2q+1-row window in LDS.
constexpr int kZlLanes = 64;

template <typename T, int Q, int AXIS, int ZT>
__global__ void __launch_bounds__(kZlLanes * ZT) k_gen_pass_zyl(const T* __restrict__ in0, const T* __restrict__ in1,
                                                                const T* __restrict__ rows, const int N,
                                                                T* __restrict__ out0, T* __restrict__ out1) {
  static_assert(AXIS == 0 || AXIS == 1, "z and y passes");
  constexpr int W = 2 * Q + 1;
  constexpr int R = (ZT + 1) * Q + 1;  // lattice rows of one block
  constexpr bool kTwo = AXIS == 1;
  __shared__ T s0[R * kZlLanes];
  __shared__ T s1[kTwo ? R * kZlLanes : 1];
  const T* __restrict__ kr = rows + (2 * AXIS) * (Q * W);
  const T* __restrict__ mr = kr + Q * W;
  const int tiles = (N + kZlLanes - 1) / kZlLanes;
  const int b = blockIdx.x;
  const int tile = b % tiles, rest = b / tiles;
  const int m = rest % N, chunk = rest / N;
  const int e0 = chunk * ZT;
  const int lane = threadIdx.x % kZlLanes, slot = threadIdx.x / kZlLanes;
  const int i = tile * kZlLanes + lane;
  const bool live = i < N;
  const int64_t step = AXIS == 0 ? static_cast<int64_t>(N) * N : N;  // along the line
  const int64_t base = (AXIS == 0 ? static_cast<int64_t>(m) * N : static_cast<int64_t>(m) * N * N) + i;
  if (live) {
    for (int r = slot; r < R; r += ZT) {
      const int64_t at = base + static_cast<int64_t>(wrap(e0 * Q - Q + r, N)) * step;
      s0[r * kZlLanes + lane] = in0[at];
      if constexpr (kTwo) s1[r * kZlLanes + lane] = in1[at];
    }
  }
  __syncthreads();
  if (!live) return;
  T w0[W], w1[kTwo ? W : 1];
#pragma unroll
  for (int u = 0; u < W; ++u) {
    w0[u] = s0[(slot * Q + u) * kZlLanes + lane];
    if constexpr (kTwo) w1[u] = s1[(slot * Q + u) * kZlLanes + lane];
  }
  const int e = e0 + slot;
#pragma unroll
  for (int c = 0; c < Q; ++c) {
    T a0 = T(0), a1 = T(0);
#pragma unroll
    for (int o = -Q; o <= Q; ++o) {
      if (c != 0 && (o < -c || o > Q - c)) continue;  // structural zero of row c
      const T kv = kr[c * W + o + Q], mv = mr[c * W + o + Q];
      const T v0 = w0[c + o + Q];
      a0 = fma(mv, v0, a0);
      a1 = fma(kv, v0, a1);
      if constexpr (kTwo) a1 = fma(mv, w1[c + o + Q], a1);
    }
    const int64_t at = base + static_cast<int64_t>(e * Q + c) * step;
    out0[at] = a0;
    out1[at] = a1;
  }
}

// The x pass for order Q with its epilogue, in the same form: a thread takes one element
// segment of an x row (loads at a stride of Q values across the wavefront, each thread's
// window contiguous), y = Kx U1 + Mx V, then the apply, residual or smoother-step epilogue.
template <typename T, int Q, int EPI>
__global__ void __launch_bounds__(kGB) k_gen_pass_x(const T* __restrict__ in0, const T* __restrict__ in1,
                                                     const T* __restrict__ rows, const T* __restrict__ dinv,
                                                     const int N, T* __restrict__ out, const T* __restrict__ x,
                                                     const T* __restrict__ b, const T* xp, const T c1, const T c2) {
  constexpr int W = 2 * Q + 1;
  const T* __restrict__ kr = rows + 4 * (Q * W);
  const T* __restrict__ mr = kr + Q * W;
  const int nE = N / Q;
  const int64_t total = static_cast<int64_t>(nE) * N * N;
  const bool use_xp = xp != nullptr && c1 != T(0);
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int e, j, k;
    split3(t, nE, N, e, j, k);
    const int64_t row = (static_cast<int64_t>(k) * N + j) * N;
    T u0[W], v0[W];
#pragma unroll
    for (int u = 0; u < W; ++u) {
      const int64_t at = row + wrap(e * Q - Q + u, N);
      u0[u] = in0[at];
      v0[u] = in1[at];
    }
    const int cyz = Q * ((j % Q) + Q * (k % Q));
#pragma unroll
    for (int c = 0; c < Q; ++c) {
      T s0 = T(0);
#pragma unroll
      for (int o = -Q; o <= Q; ++o) {
        if (c != 0 && (o < -c || o > Q - c)) continue;  // structural zero of row c
        s0 = fma(kr[c * W + o + Q], u0[c + o + Q], s0);
        s0 = fma(mr[c * W + o + Q], v0[c + o + Q], s0);
      }
      const int64_t at = row + e * Q + c;
      if constexpr (EPI == static_cast<int>(Epi::Apply)) {
        out[at] = s0;
      } else if constexpr (EPI == static_cast<int>(Epi::Residual)) {
        out[at] = b[at] - s0;
      } else {  // Epi::Cheb, x_prev read as 0 when absent
        const T xv = x[at];
        const T xpv = use_xp ? xp[at] : T(0);
        out[at] = xv + c1 * (xv - xpv) + c2 * dinv[c + cyz] * (b[at] - s0);
      }
    }
  }
}

// The x pass for order Q staged through LDS: a block loads kXlSegs / (N / Q) whole x rows of
// U1 and V with coalesced loads (element e of a row at slot e S, S = Q or Q + 1 whichever is
// odd, so that a wavefront reading one window position of consecutive elements hits distinct
// banks), each thread takes one element segment and keeps its Q sums in registers, writes them
// over U1 once every window is read, and the epilogue then runs a thread per node with
// coalesced reads of x, b and x_prev.  N / Q must divide kXlSegs.
constexpr int kXlSegs = 256;

template <int Q>
constexpr int xl_stride() {
  return (Q & 1) ? Q : Q + 1;
}

template <typename T, int Q, int EPI>
__global__ void __launch_bounds__(kXlSegs) k_gen_pass_xl(const T* __restrict__ in0, const T* __restrict__ in1,
                                                          const T* __restrict__ rows, const T* __restrict__ dinv,
                                                          const int N, T* __restrict__ out,
                                                          const T* __restrict__ x, const T* __restrict__ b,
                                                          const T* xp, const T c1, const T c2) {
  constexpr int W = 2 * Q + 1;
  constexpr int S = xl_stride<Q>();
  const T* __restrict__ kr = rows + 4 * (Q * W);
  const T* __restrict__ mr = kr + Q * W;
  const int nE = N / Q;
  const int R = kXlSegs / nE;      // x rows per block
  const int rowlen = nE * S;       // LDS values per row and array
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* su = reinterpret_cast<T*>(smem_raw);  // [R][rowlen] U1, then the sums
  T* sv = su + R * rowlen;                  // V
  const int64_t nrows = static_cast<int64_t>(N) * N;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * R;
  const int rows_here = static_cast<int>(nrows - row0 < R ? nrows - row0 : R);
  const int tid = threadIdx.x;
  const int64_t base = row0 * N;
  // node a of row r sits at slot r rowlen + (a / Q) S + a % Q, which is (v / Q) S + v % Q for
  // v = r N + a (N = nE Q, rowlen = nE S): the apply and the residual take that form (measured
  // faster), the smoother step the row split (measured faster there)
  constexpr bool kFlat = EPI != static_cast<int>(Epi::Cheb);
  for (int v = tid; v < rows_here * N; v += kXlSegs) {
    int slot;
    if constexpr (kFlat) {
      slot = (v / Q) * S + (v % Q);
    } else {
      const int r = v / N, a = v - r * N;
      slot = r * rowlen + (a / Q) * S + (a % Q);
    }
    su[slot] = in0[base + v];
    sv[slot] = in1[base + v];
  }
  __syncthreads();
  const int r = tid / nE, e = tid - r * nE;
  const bool live = r < rows_here;
  T s0[Q];
  if (live) {
    const int el = e == 0 ? nE - 1 : e - 1, er = e == nE - 1 ? 0 : e + 1;
    const T* ru = su + r * rowlen;
    const T* rv = sv + r * rowlen;
    T u0[W], v0[W];
#pragma unroll
    for (int c = 0; c < Q; ++c) {
      u0[c] = ru[el * S + c];
      v0[c] = rv[el * S + c];
      u0[Q + c] = ru[e * S + c];
      v0[Q + c] = rv[e * S + c];
    }
    u0[2 * Q] = ru[er * S];
    v0[2 * Q] = rv[er * S];
#pragma unroll
    for (int c = 0; c < Q; ++c) {
      T acc = T(0);
#pragma unroll
      for (int o = -Q; o <= Q; ++o) {
        if (c != 0 && (o < -c || o > Q - c)) continue;  // structural zero of row c
        acc = fma(kr[c * W + o + Q], u0[c + o + Q], acc);
        acc = fma(mr[c * W + o + Q], v0[c + o + Q], acc);
      }
      s0[c] = acc;
    }
  }
  __syncthreads();
  if (live) {
#pragma unroll
    for (int c = 0; c < Q; ++c) su[r * rowlen + e * S + c] = s0[c];
  }
  __syncthreads();
  const bool use_xp = xp != nullptr && c1 != T(0);
  for (int v = tid; v < rows_here * N; v += kXlSegs) {
    const int rr = kFlat ? 0 : v / N, a = kFlat ? v : v - rr * N;
    const int64_t at = base + v;
    const T y = su[rr * rowlen + (a / Q) * S + (a % Q)];
    if constexpr (EPI == static_cast<int>(Epi::Apply)) {
      out[at] = y;
    } else if constexpr (EPI == static_cast<int>(Epi::Residual)) {
      out[at] = b[at] - y;
    } else {  // Epi::Cheb, x_prev read as 0 when absent
      const int64_t row = row0 + rr;
      const int j = static_cast<int>(row % N), k = static_cast<int>(row / N);
      const T xv = x[at];
      const T xpv = use_xp ? xp[at] : T(0);
      out[at] = xv + c1 * (xv - xpv) + c2 * dinv[(a % Q) + Q * ((j % Q) + Q * (k % Q))] * (b[at] - y);
    }
  }
}

// false when N / Q does not divide kXlSegs (the caller takes the register form)
template <typename T, int Q, int EPI>
bool gen_xl_launch(const T* t3, const T* t4, const T* rows, const T* dinv, const ApplyArgs& a, hipStream_t s,
                   hipError_t* err) {
  const int N = a.N;
  const int nE = N / Q;
  if (nE > kXlSegs || kXlSegs % nE != 0) return false;
  const int R = kXlSegs / nE;
  const size_t lds = sizeof(T) * 2 * static_cast<size_t>(R) * nE * xl_stride<Q>();
  if (lds > 65536) {
    const void* fn = reinterpret_cast<const void*>(&k_gen_pass_xl<T, Q, EPI>);
    *err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (*err != hipSuccess) return true;
  }
  const int64_t nrows = static_cast<int64_t>(N) * N;
  const dim3 g(static_cast<unsigned>((nrows + R - 1) / R)), bl(kXlSegs);
  hipLaunchKernelGGL((k_gen_pass_xl<T, Q, EPI>), g, bl, lds, s, t3, t4, rows, dinv, N, static_cast<T*>(a.out),
                     static_cast<const T*>(a.x), static_cast<const T*>(a.b), static_cast<const T*>(a.xp),
                     static_cast<T>(a.c1), static_cast<T>(a.c2));
  *err = hipGetLastError();
  return true;
}

// the x pass of order Q in the LDS or the per-element form; false when neither applies
template <typename T, int Q>
bool gen_x_q(const T* t3, const T* t4, const T* rows, const T* dinv, const ApplyArgs& a, hipStream_t s,
             hipError_t* err) {
  if (gen_x_lds(Q, a.epi)) {
    switch (a.epi) {
      case Epi::Apply:
        if (gen_xl_launch<T, Q, static_cast<int>(Epi::Apply)>(t3, t4, rows, dinv, a, s, err)) return true;
        break;
      case Epi::Residual:
        if (gen_xl_launch<T, Q, static_cast<int>(Epi::Residual)>(t3, t4, rows, dinv, a, s, err)) return true;
        break;
      case Epi::Cheb:
        if (gen_xl_launch<T, Q, static_cast<int>(Epi::Cheb)>(t3, t4, rows, dinv, a, s, err)) return true;
        break;
      default:
        break;
    }
  }
  if (!gen_x_per_element(Q, a.epi)) return false;
  const int N = a.N;
  const dim3 g(gen_grid(static_cast<int64_t>(N / Q) * N * N)), bl(kGB);
  const T* x = static_cast<const T*>(a.x);
  const T* b = static_cast<const T*>(a.b);
  const T* xp = static_cast<const T*>(a.xp);
  T* out = static_cast<T*>(a.out);
  switch (a.epi) {
    case Epi::Apply:
      hipLaunchKernelGGL((k_gen_pass_x<T, Q, static_cast<int>(Epi::Apply)>), g, bl, 0, s, t3, t4, rows, dinv, N, out,
                         x, b, xp, T(0), T(0));
      break;
    case Epi::Residual:
      hipLaunchKernelGGL((k_gen_pass_x<T, Q, static_cast<int>(Epi::Residual)>), g, bl, 0, s, t3, t4, rows, dinv, N,
                         out, x, b, xp, T(0), T(0));
      break;
    case Epi::Cheb:
      hipLaunchKernelGGL((k_gen_pass_x<T, Q, static_cast<int>(Epi::Cheb)>), g, bl, 0, s, t3, t4, rows, dinv, N, out,
                         x, b, xp, static_cast<T>(a.c1), static_cast<T>(a.c2));
      break;
    default:
      *err = hipErrorInvalidValue;
      return true;
  }
  *err = hipGetLastError();
  return true;
}

// false for an order without a generic instance or a pass left to the per-node form
template <typename T>
bool gen_x(int q, const T* t3, const T* t4, const T* rows, const T* dinv, const ApplyArgs& a, hipStream_t s,
           hipError_t* err) {
  switch (q) {
    case 3: return gen_x_q<T, 3>(t3, t4, rows, dinv, a, s, err);
    case 5: return gen_x_q<T, 5>(t3, t4, rows, dinv, a, s, err);
    case 6: return gen_x_q<T, 6>(t3, t4, rows, dinv, a, s, err);
    case 7: return gen_x_q<T, 7>(t3, t4, rows, dinv, a, s, err);
    case 8: return gen_x_q<T, 8>(t3, t4, rows, dinv, a, s, err);
    case 9: return gen_x_q<T, 9>(t3, t4, rows, dinv, a, s, err);
    case 10: return gen_x_q<T, 10>(t3, t4, rows, dinv, a, s, err);
    case 11: return gen_x_q<T, 11>(t3, t4, rows, dinv, a, s, err);
    case 12: return gen_x_q<T, 12>(t3, t4, rows, dinv, a, s, err);
    case 13: return gen_x_q<T, 13>(t3, t4, rows, dinv, a, s, err);
    case 14: return gen_x_q<T, 14>(t3, t4, rows, dinv, a, s, err);
    case 15: return gen_x_q<T, 15>(t3, t4, rows, dinv, a, s, err);
    case 16: return gen_x_q<T, 16>(t3, t4, rows, dinv, a, s, err);
  }
  return false;
}

template <typename T, int Q, int C>
void gen_zy_qc(const T* x, const T* rows, int N, T* t1, T* t2, T* t3, T* t4, hipStream_t s) {
  const dim3 g(gen_grid(static_cast<int64_t>(N / Q / C) * N * N)), bl(kGB);
  hipLaunchKernelGGL((k_gen_pass_zy<T, Q, 0, C>), g, bl, 0, s, x, nullptr, rows, N, t1, t2);
  hipLaunchKernelGGL((k_gen_pass_zy<T, Q, 1, C>), g, bl, 0, s, static_cast<const T*>(t1), static_cast<const T*>(t2),
                     rows, N, t3, t4);
}

// Two elements per thread pay where that instance keeps at least the occupancy of the one-element
// instance in both passes (the register count decides; measured near 256^3 DoFs: FP32 q = 8 apply
// 230 -> 175 us, solve 35.8 -> 31.7 ms), and cost up to 7 % of a solve where it lowers it (fewer
// waves to hide the strided loads, and half the threads on the coarse levels).
template <typename T, int Q>
bool zy_two_pays() {
  static const bool pays = [] {
    auto occ = [](const void* f) {
      int n = 0;
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kGB, 0) == hipSuccess ? n : -1;
    };
    const int z1 = occ(reinterpret_cast<const void*>(&k_gen_pass_zy<T, Q, 0, 1>));
    const int y1 = occ(reinterpret_cast<const void*>(&k_gen_pass_zy<T, Q, 1, 1>));
    const int z2 = occ(reinterpret_cast<const void*>(&k_gen_pass_zy<T, Q, 0, 2>));
    const int y2 = occ(reinterpret_cast<const void*>(&k_gen_pass_zy<T, Q, 1, 2>));
    return z1 > 0 && y1 > 0 && z2 >= z1 && y2 >= y1;
  }();
  return pays;
}

template <typename T, int Q, int ZT>
void gen_zy_ql(const T* x, const T* rows, int N, T* t1, T* t2, T* t3, T* t4, hipStream_t s) {
  const int tiles = (N + kZlLanes - 1) / kZlLanes;
  const dim3 g(static_cast<unsigned>(tiles * N * (N / Q / ZT))), bl(kZlLanes * ZT);
  hipLaunchKernelGGL((k_gen_pass_zyl<T, Q, 0, ZT>), g, bl, 0, s, x, nullptr, rows, N, t1, t2);
  hipLaunchKernelGGL((k_gen_pass_zyl<T, Q, 1, ZT>), g, bl, 0, s, static_cast<const T*>(t1),
                     static_cast<const T*>(t2), rows, N, t3, t4);
}

// The z and y passes: two element segments per thread where that pays (above), else staged
// through LDS on levels of at least 128 nodes a side (FP64: up to q = 10, where a block's LDS
// stays within 32 KB), else one segment per thread.  Measured near 256^3 DoFs against the
// one-segment form, the LDS form takes FP32-cycle solves 9 % (q = 14) and 4 % (q = 16) faster;
// on narrower levels a 64-lane tile runs partly empty and it lost up to 9 % of a solve (q = 5),
// and in FP64 at q = 14, 16 (1.5 waves per SIMD at 50 KB per block) the apply lost 12-17 %.
template <typename T, int Q>
void gen_zy_q(const T* x, const T* rows, int N, T* t1, T* t2, T* t3, T* t4, hipStream_t s) {
  constexpr int ZT = sizeof(T) == 4 ? 4 : 2;
  if ((N / Q) % 2 == 0 && zy_two_pays<T, Q>()) {
    gen_zy_qc<T, Q, 2>(x, rows, N, t1, t2, t3, t4, s);
    return;
  }
  if constexpr (sizeof(T) == 4 || Q <= 10) {
    if (N >= 128 && (N / Q) % ZT == 0) {
      gen_zy_ql<T, Q, ZT>(x, rows, N, t1, t2, t3, t4, s);
      return;
    }
  }
  gen_zy_qc<T, Q, 1>(x, rows, N, t1, t2, t3, t4, s);
}

// z and y passes by order (false for an order without a generic instance)
template <typename T>
bool gen_zy(int q, const T* x, const T* rows, int N, T* t1, T* t2, T* t3, T* t4, hipStream_t s) {
  switch (q) {
    case 3: gen_zy_q<T, 3>(x, rows, N, t1, t2, t3, t4, s); return true;
    case 5: gen_zy_q<T, 5>(x, rows, N, t1, t2, t3, t4, s); return true;
    case 6: gen_zy_q<T, 6>(x, rows, N, t1, t2, t3, t4, s); return true;
    case 7: gen_zy_q<T, 7>(x, rows, N, t1, t2, t3, t4, s); return true;
    case 8: gen_zy_q<T, 8>(x, rows, N, t1, t2, t3, t4, s); return true;
    case 9: gen_zy_q<T, 9>(x, rows, N, t1, t2, t3, t4, s); return true;
    case 10: gen_zy_q<T, 10>(x, rows, N, t1, t2, t3, t4, s); return true;
    case 11: gen_zy_q<T, 11>(x, rows, N, t1, t2, t3, t4, s); return true;
    case 12: gen_zy_q<T, 12>(x, rows, N, t1, t2, t3, t4, s); return true;
    case 13: gen_zy_q<T, 13>(x, rows, N, t1, t2, t3, t4, s); return true;
    case 14: gen_zy_q<T, 14>(x, rows, N, t1, t2, t3, t4, s); return true;
    case 15: gen_zy_q<T, 15>(x, rows, N, t1, t2, t3, t4, s); return true;
    case 16: gen_zy_q<T, 16>(x, rows, N, t1, t2, t3, t4, s); return true;
  }
  return false;
}

template <typename T>
hipError_t gen_apply_t(const GenOp& op, const ApplyArgs& a, void* t1, void* t2, void* t3, void* t4, hipStream_t s) {
  const int N = a.N, q = op.q;
  const int64_t n3 = static_cast<int64_t>(N) * N * N;
  const T* rows = static_cast<const T*>(sizeof(T) == 4 ? static_cast<const void*>(op.rows32) : op.rows64);
  const T* dinv = static_cast<const T*>(sizeof(T) == 4 ? static_cast<const void*>(op.dinv32) : op.dinv64);
  const dim3 g(gen_grid(n3)), bl(kGB);
  if (!gen_zy<T>(q, static_cast<const T*>(a.x), rows, N, static_cast<T*>(t1), static_cast<T*>(t2),
                 static_cast<T*>(t3), static_cast<T*>(t4), s)) {
    hipLaunchKernelGGL((k_gen_pass<T, 0, 0>), g, bl, 0, s, static_cast<const T*>(a.x), nullptr, rows, dinv, q, N,
                       static_cast<T*>(t1), static_cast<T*>(t2), nullptr, nullptr, nullptr, T(0), T(0));
    hipLaunchKernelGGL((k_gen_pass<T, 1, 0>), g, bl, 0, s, static_cast<const T*>(t1), static_cast<const T*>(t2),
                       rows, dinv, q, N, static_cast<T*>(t3), static_cast<T*>(t4), nullptr, nullptr, nullptr, T(0),
                       T(0));
  }
  {
    hipError_t e = hipSuccess;
    if (gen_x<T>(q, static_cast<const T*>(t3), static_cast<const T*>(t4), rows, dinv, a, s, &e)) return e;
  }
  const T* x = static_cast<const T*>(a.x);
  const T* b = static_cast<const T*>(a.b);
  T* out = static_cast<T*>(a.out);
  switch (a.epi) {
    case Epi::Apply:
      hipLaunchKernelGGL((k_gen_pass<T, 2, static_cast<int>(Epi::Apply)>), g, bl, 0, s, static_cast<const T*>(t3),
                         static_cast<const T*>(t4), rows, dinv, q, N, out, nullptr, x, b,
                         static_cast<const T*>(a.xp), T(0), T(0));
      break;
    case Epi::Residual:
      hipLaunchKernelGGL((k_gen_pass<T, 2, static_cast<int>(Epi::Residual)>), g, bl, 0, s,
                         static_cast<const T*>(t3), static_cast<const T*>(t4), rows, dinv, q, N, out, nullptr, x, b,
                         static_cast<const T*>(a.xp), T(0), T(0));
      break;
    case Epi::Cheb:
      hipLaunchKernelGGL((k_gen_pass<T, 2, static_cast<int>(Epi::Cheb)>), g, bl, 0, s, static_cast<const T*>(t3),
                         static_cast<const T*>(t4), rows, dinv, q, N, out, nullptr, x, b,
                         static_cast<const T*>(a.xp), static_cast<T>(a.c1), static_cast<T>(a.c2));
      break;
    default:
      return hipErrorInvalidValue;  // the fused variants exist for q = 1, 2, 4 only
  }
  return hipGetLastError();
}

// ---- transfers: P1 and P1^T along one axis, a thread per output node
// p: 2q x (q+1) (fine node 2qE + b from coarse q E + a), r: q x (4q+1) (coarse node
// q E + a from fine 2qE - 2q + t); extents: (X, Y, Z) of the output, the input equal
// except along AXIS
template <typename T, int AXIS, bool ACC>
__global__ void __launch_bounds__(kGB) k_gen_prolong(const T* __restrict__ in, T* __restrict__ out,
                                                      const double* __restrict__ p, const int q, const int X,
                                                      const int Y, const int Z, const int Nc) {
  const int64_t total = static_cast<int64_t>(X) * Y * Z;
  const int ix = AXIS == 0 ? Nc : X, iy = AXIS == 1 ? Nc : Y;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int i, j, k;
    split3(idx, X, Y, i, j, k);
    const int f = AXIS == 0 ? i : (AXIS == 1 ? j : k);
    const int E = f / (2 * q), bb = f - 2 * q * E;
    double s = 0.0;
    for (int a = 0; a <= q; ++a) {
      const int cc = wrap(q * E + a, Nc);
      int ii = i, jj = j, kk = k;
      if (AXIS == 0) ii = cc;
      else if (AXIS == 1) jj = cc;
      else kk = cc;
      s = fma(p[bb * (q + 1) + a], static_cast<double>(in[(static_cast<int64_t>(kk) * iy + jj) * ix + ii]), s);
    }
    out[idx] = ACC ? static_cast<T>(static_cast<double>(out[idx]) + s) : static_cast<T>(s);
  }
}

template <typename T, int AXIS>
__global__ void __launch_bounds__(kGB) k_gen_restrict(const T* __restrict__ in, T* __restrict__ out,
                                                       const double* __restrict__ r, const int q, const int X,
                                                       const int Y, const int Z, const int Nf) {
  const int64_t total = static_cast<int64_t>(X) * Y * Z;
  const int ix = AXIS == 0 ? Nf : X, iy = AXIS == 1 ? Nf : Y;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < total;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int i, j, k;
    split3(idx, X, Y, i, j, k);
    const int c = AXIS == 0 ? i : (AXIS == 1 ? j : k);
    const int E = c / q, a = c - q * E;
    double s = 0.0;
    for (int t = 0; t <= 4 * q; ++t) {
      const double w = r[a * (4 * q + 1) + t];
      if (w == 0.0) continue;
      const int ff = wrap(2 * q * E - 2 * q + t, Nf);
      int ii = i, jj = j, kk = k;
      if (AXIS == 0) ii = ff;
      else if (AXIS == 1) jj = ff;
      else kk = ff;
      s = fma(w, static_cast<double>(in[(static_cast<int64_t>(kk) * iy + jj) * ix + ii]), s);
    }
    out[idx] = static_cast<T>(s);
  }
}

// The transfers of order Q along one axis, a thread per coarse element of a lattice line (lanes
// along x for the y and z axes, so their loads and stores are coalesced): the prolongation loads
// the element's q+1 coarse values once and writes its 2q fine nodes, the restriction loads the
// 4q+1 fine values the element's rows reach once and writes its q coarse nodes.  Same weights,
// FP64 accumulation and tap order as the thread-per-node kernels above.  X, Y, Z: extents of the
// output; the input's extent along AXIS is Nc (prolongation) or Nf (restriction).
template <int AXIS>
__device__ inline void xfer_line(int64_t t, int nE, int X, int Y, int& i, int& j, int& k, int& E) {
  if constexpr (AXIS == 0) { split3(t, nE, Y, E, j, k); i = 0; }
  else if constexpr (AXIS == 1) { split3(t, X, nE, i, E, k); j = 0; }
  else { split3(t, X, Y, i, j, E); k = 0; }
}

template <typename T, int Q, int AXIS, bool ACC>
__global__ void __launch_bounds__(kGB) k_gen_prolong_e(const T* __restrict__ in, T* __restrict__ out,
                                                        const double* __restrict__ p, const int X, const int Y,
                                                        const int Z, const int Nc) {
  const int nE = Nc / Q;
  const int ix = AXIS == 0 ? Nc : X, iy = AXIS == 1 ? Nc : Y;
  const int64_t total = static_cast<int64_t>(nE) * (AXIS == 0 ? 1 : X) * (AXIS == 1 ? 1 : Y) * (AXIS == 2 ? 1 : Z);
  const int64_t sin = AXIS == 0 ? 1 : (AXIS == 1 ? ix : static_cast<int64_t>(ix) * iy);
  const int64_t sout = AXIS == 0 ? 1 : (AXIS == 1 ? X : static_cast<int64_t>(X) * Y);
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int i, j, k, E;
    xfer_line<AXIS>(t, nE, X, Y, i, j, k, E);
    const int64_t bin = (static_cast<int64_t>(k) * iy + j) * ix + i;
    const int64_t bout = (static_cast<int64_t>(k) * Y + j) * X + i;
    double v[Q + 1];
#pragma unroll
    for (int a = 0; a <= Q; ++a) v[a] = static_cast<double>(in[bin + wrap(Q * E + a, Nc) * sin]);
#pragma unroll
    for (int bb = 0; bb < 2 * Q; ++bb) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a <= Q; ++a) s = fma(p[bb * (Q + 1) + a], v[a], s);
      const int64_t at = bout + static_cast<int64_t>(2 * Q * E + bb) * sout;
      out[at] = ACC ? static_cast<T>(static_cast<double>(out[at]) + s) : static_cast<T>(s);
    }
  }
}

template <typename T, int Q, int AXIS>
__global__ void __launch_bounds__(kGB) k_gen_restrict_e(const T* __restrict__ in, T* __restrict__ out,
                                                         const double* __restrict__ r, const int X, const int Y,
                                                         const int Z, const int Nf) {
  constexpr int W = 4 * Q + 1;
  const int Nc = Nf / 2, nE = Nc / Q;
  const int ix = AXIS == 0 ? Nf : X, iy = AXIS == 1 ? Nf : Y;
  const int64_t total = static_cast<int64_t>(nE) * (AXIS == 0 ? 1 : X) * (AXIS == 1 ? 1 : Y) * (AXIS == 2 ? 1 : Z);
  const int64_t sin = AXIS == 0 ? 1 : (AXIS == 1 ? ix : static_cast<int64_t>(ix) * iy);
  const int64_t sout = AXIS == 0 ? 1 : (AXIS == 1 ? X : static_cast<int64_t>(X) * Y);
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int i, j, k, E;
    xfer_line<AXIS>(t, nE, X, Y, i, j, k, E);
    const int64_t bin = (static_cast<int64_t>(k) * iy + j) * ix + i;
    const int64_t bout = (static_cast<int64_t>(k) * Y + j) * X + i;
    T w[W];
#pragma unroll
    for (int u = 0; u < W; ++u) w[u] = in[bin + wrap(2 * Q * E - 2 * Q + u, Nf) * sin];
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      double s = 0.0;
#pragma unroll
      for (int u = a == 0 ? 0 : 2 * Q; u < W; ++u) {  // an interior node's rows stop at its element
        const double wt = r[a * W + u];
        if (wt != 0.0) s = fma(wt, static_cast<double>(w[u]), s);
      }
      out[bout + static_cast<int64_t>(Q * E + a) * sout] = static_cast<T>(s);
    }
  }
}

template <typename T, int Q>
void gen_prolong_q(const double* p, const T* ec, T* t1, T* t2, T* uf, int Nc, hipStream_t s) {
  const int Nf = 2 * Nc, nE = Nc / Q;
  const dim3 bl(kGB);
  hipLaunchKernelGGL((k_gen_prolong_e<T, Q, 0, false>), dim3(gen_grid(static_cast<int64_t>(nE) * Nc * Nc)), bl, 0,
                     s, ec, t1, p, Nf, Nc, Nc, Nc);
  hipLaunchKernelGGL((k_gen_prolong_e<T, Q, 1, false>), dim3(gen_grid(static_cast<int64_t>(nE) * Nf * Nc)), bl, 0,
                     s, static_cast<const T*>(t1), t2, p, Nf, Nf, Nc, Nc);
  hipLaunchKernelGGL((k_gen_prolong_e<T, Q, 2, true>), dim3(gen_grid(static_cast<int64_t>(nE) * Nf * Nf)), bl, 0,
                     s, static_cast<const T*>(t2), uf, p, Nf, Nf, Nf, Nc);
}

template <typename T, int Q>
void gen_restrict_q(const double* r, const T* rf, T* t1, T* t2, T* rc, int Nc, hipStream_t s) {
  const int Nf = 2 * Nc, nE = Nc / Q;
  const dim3 bl(kGB);
  hipLaunchKernelGGL((k_gen_restrict_e<T, Q, 0>), dim3(gen_grid(static_cast<int64_t>(nE) * Nf * Nf)), bl, 0, s,
                     rf, t1, r, Nc, Nf, Nf, Nf);
  hipLaunchKernelGGL((k_gen_restrict_e<T, Q, 1>), dim3(gen_grid(static_cast<int64_t>(nE) * Nc * Nf)), bl, 0, s,
                     static_cast<const T*>(t1), t2, r, Nc, Nc, Nf, Nf);
  hipLaunchKernelGGL((k_gen_restrict_e<T, Q, 2>), dim3(gen_grid(static_cast<int64_t>(nE) * Nc * Nc)), bl, 0, s,
                     static_cast<const T*>(t2), rc, r, Nc, Nc, Nc, Nf);
}

// the per-element transfers by order (false for an order without an instance)
template <typename T>
bool gen_xfer_e(bool prolong, int q, const double* w, const T* in, T* t1, T* t2, T* out, int Nc, hipStream_t s) {
#define GMG_XFER_CASE(QQ)                                                  \
  case QQ:                                                                 \
    if (prolong) gen_prolong_q<T, QQ>(w, in, t1, t2, out, Nc, s);          \
    else gen_restrict_q<T, QQ>(w, in, t1, t2, out, Nc, s);                 \
    return true;
  switch (q) {
    GMG_XFER_CASE(3)
    GMG_XFER_CASE(5)
    GMG_XFER_CASE(6)
    GMG_XFER_CASE(7)
    GMG_XFER_CASE(8)
    GMG_XFER_CASE(9)
    GMG_XFER_CASE(10)
    GMG_XFER_CASE(11)
    GMG_XFER_CASE(12)
    GMG_XFER_CASE(13)
    GMG_XFER_CASE(14)
    GMG_XFER_CASE(15)
    GMG_XFER_CASE(16)
  }
#undef GMG_XFER_CASE
  return false;
}

template <typename T>
hipError_t gen_prolong_t(const GenXfer& t, const T* ec, T* t1, T* t2, T* uf, int Nc, hipStream_t s) {
  if (gen_xfer_e<T>(true, t.q, t.p, ec, t1, t2, uf, Nc, s)) return hipGetLastError();
  const int Nf = 2 * Nc, q = t.q;
  const dim3 bl(kGB);
  hipLaunchKernelGGL((k_gen_prolong<T, 0, false>), dim3(gen_grid(static_cast<int64_t>(Nf) * Nc * Nc)), bl, 0, s, ec,
                     t1, t.p, q, Nf, Nc, Nc, Nc);
  hipLaunchKernelGGL((k_gen_prolong<T, 1, false>), dim3(gen_grid(static_cast<int64_t>(Nf) * Nf * Nc)), bl, 0, s,
                     static_cast<const T*>(t1), t2, t.p, q, Nf, Nf, Nc, Nc);
  hipLaunchKernelGGL((k_gen_prolong<T, 2, true>), dim3(gen_grid(static_cast<int64_t>(Nf) * Nf * Nf)), bl, 0, s,
                     static_cast<const T*>(t2), uf, t.p, q, Nf, Nf, Nf, Nc);
  return hipGetLastError();
}

template <typename T>
hipError_t gen_restrict_t(const GenXfer& t, const T* rf, T* t1, T* t2, T* rc, int Nc, hipStream_t s) {
  if (gen_xfer_e<T>(false, t.q, t.r, rf, t1, t2, rc, Nc, s)) return hipGetLastError();
  const int Nf = 2 * Nc, q = t.q;
  const dim3 bl(kGB);
  hipLaunchKernelGGL((k_gen_restrict<T, 0>), dim3(gen_grid(static_cast<int64_t>(Nc) * Nf * Nf)), bl, 0, s, rf, t1,
                     t.r, q, Nc, Nf, Nf, Nf);
  hipLaunchKernelGGL((k_gen_restrict<T, 1>), dim3(gen_grid(static_cast<int64_t>(Nc) * Nc * Nf)), bl, 0, s,
                     static_cast<const T*>(t1), t2, t.r, q, Nc, Nc, Nf, Nf);
  hipLaunchKernelGGL((k_gen_restrict<T, 2>), dim3(gen_grid(static_cast<int64_t>(Nc) * Nc * Nc)), bl, 0, s,
                     static_cast<const T*>(t2), rc, t.r, q, Nc, Nc, Nc, Nf);
  return hipGetLastError();
}

// ---- node-class arithmetic with the class table in device memory (q^3 values)
template <typename T>
__global__ void __launch_bounds__(kGB) k_gclass_scale(const double* __restrict__ tab, const int q, const int N,
                                                       const double c, const T* in, T* out) {
  const int64_t n3 = static_cast<int64_t>(N) * N * N;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < n3;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int i, j, k;
    split3(idx, N, N, i, j, k);
    const double d = tab ? tab[(i % q) + q * ((j % q) + q * (k % q))] : 1.0;
    const double v = in ? static_cast<double>(in[idx]) : 1.0;
    out[idx] = static_cast<T>(c * d * v);
  }
}

template <typename T>
__global__ void __launch_bounds__(kGB) k_gclass_axpy(const double* __restrict__ tab, const int q, const int N,
                                                      const double c, T* v) {
  const int64_t n3 = static_cast<int64_t>(N) * N * N;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < n3;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int i, j, k;
    split3(idx, N, N, i, j, k);
    v[idx] = static_cast<T>(static_cast<double>(v[idx]) + c * tab[(i % q) + q * ((j % q) + q * (k % q))]);
  }
}

// per-block partials of sum tab[class(i)] x_i, in a fixed order
template <typename T>
__global__ void __launch_bounds__(kGB) k_gclass_dot(const double* __restrict__ tab, const int q, const int N,
                                                     const T* __restrict__ x, double* part) {
  __shared__ double red[kGB / 64];
  const int64_t n3 = static_cast<int64_t>(N) * N * N;
  double s = 0.0;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; idx < n3;
       idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    int i, j, k;
    split3(idx, N, N, i, j, k);
    s = fma(tab[(i % q) + q * ((j % q) + q * (k % q))], static_cast<double>(x[idx]), s);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kGB / 64; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

}  // namespace

hipError_t launch_gen_apply(const GenOp& op, bool fp32, const ApplyArgs& a, void* const tmp[4], hipStream_t s) {
  if (op.q < 1 || op.q > kGenMaxQ || a.N != op.q * a.n || a.N < 1) return hipErrorInvalidValue;
  if (fp32) return gen_apply_t<float>(op, a, tmp[0], tmp[1], tmp[2], tmp[3], s);
  return gen_apply_t<double>(op, a, tmp[0], tmp[1], tmp[2], tmp[3], s);
}

hipError_t launch_gen_prolong(const GenXfer& t, bool fp32, const void* ec, void* t1, void* t2, void* uf, int Nc,
                              hipStream_t s) {
  if (t.q < 1 || t.q > kGenMaxQ || Nc < t.q || Nc % t.q != 0) return hipErrorInvalidValue;
  if (fp32)
    return gen_prolong_t<float>(t, static_cast<const float*>(ec), static_cast<float*>(t1), static_cast<float*>(t2),
                                static_cast<float*>(uf), Nc, s);
  return gen_prolong_t<double>(t, static_cast<const double*>(ec), static_cast<double*>(t1), static_cast<double*>(t2),
                               static_cast<double*>(uf), Nc, s);
}

hipError_t launch_gen_restrict(const GenXfer& t, bool fp32, const void* rf, void* t1, void* t2, void* rc, int Nc,
                               hipStream_t s) {
  if (t.q < 1 || t.q > kGenMaxQ || Nc < t.q || Nc % t.q != 0) return hipErrorInvalidValue;
  if (fp32)
    return gen_restrict_t<float>(t, static_cast<const float*>(rf), static_cast<float*>(t1), static_cast<float*>(t2),
                                 static_cast<float*>(rc), Nc, s);
  return gen_restrict_t<double>(t, static_cast<const double*>(rf), static_cast<double*>(t1), static_cast<double*>(t2),
                                static_cast<double*>(rc), Nc, s);
}

hipError_t launch_gclass_scale(bool fp32, int q, int N, const double* tab_dev, double c, const void* in, void* out,
                               hipStream_t s) {
  const unsigned g = gen_grid(static_cast<int64_t>(N) * N * N);
  if (fp32)
    hipLaunchKernelGGL(k_gclass_scale<float>, dim3(g), dim3(kGB), 0, s, tab_dev, q, N, c,
                       static_cast<const float*>(in), static_cast<float*>(out));
  else
    hipLaunchKernelGGL(k_gclass_scale<double>, dim3(g), dim3(kGB), 0, s, tab_dev, q, N, c,
                       static_cast<const double*>(in), static_cast<double*>(out));
  return hipGetLastError();
}

hipError_t launch_gclass_axpy(int q, int N, const double* tab_dev, double c, double* v, hipStream_t s) {
  hipLaunchKernelGGL(k_gclass_axpy<double>, dim3(gen_grid(static_cast<int64_t>(N) * N * N)), dim3(kGB), 0, s,
                     tab_dev, q, N, c, v);
  return hipGetLastError();
}

hipError_t launch_gclass_dot(bool fp32, int q, int N, const double* tab_dev, const void* x, double* part,
                             int64_t part_cap, double* dst, hipStream_t s) {
  int g = static_cast<int>(gen_grid(static_cast<int64_t>(N) * N * N));
  if (g > kRedBlocks) g = kRedBlocks;
  if (part_cap < g) return hipErrorInvalidValue;
  if (fp32)
    hipLaunchKernelGGL(k_gclass_dot<float>, dim3(g), dim3(kGB), 0, s, tab_dev, q, N, static_cast<const float*>(x),
                       part);
  else
    hipLaunchKernelGGL(k_gclass_dot<double>, dim3(g), dim3(kGB), 0, s, tab_dev, q, N, static_cast<const double*>(x),
                       part);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sum_partials(part, g, part_cap, dst, s);
}

}  // namespace gmg
