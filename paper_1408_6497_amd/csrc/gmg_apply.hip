// Matrix-free, sum-factorized Q_q stiffness apply on uniform periodic meshes
// (Section 2.3.2: tensorized LGL nodal basis, so the element MatVec costs
// O(q^4) instead of O(q^6); here the tensor structure is used globally and
// every node is touched once per 1D pass).
//
// Operator:  A = Kx (x) My (x) Mz + Mx (x) Ky (x) Mz + Mx (x) My (x) Kz
// split per z plane:  g = (Kx My + Mx Ky) x,  h = Mx My x,  A x = Mz g + Kz h.
//
// Two kernels:
//
// k_apply_col (levels with N >= 64): streams z planes.
//   * a tile is 4 G full x-rows by a chunk of TZ element layers; thread (tx, ty)
//     owns one element column in x (q nodes, moved as one q-wide vector, so a
//     wavefront reads 64 q consecutive values per row) and RY rows of the 4
//     rows 4 ty .. 4 ty + 3 of the tile.  RY = 4 (one workgroup per tile),
//     except FP64 q = 4 and the FP64 q = 2 smoother steps, whose accumulators
//     do not fit the register file four rows deep, and the FP32 q = 2 residuals
//     and smoother steps, which need the occupancy of the smaller register
//     count: there RY = 2 and two workgroups share a tile, one taking rows 0, 1
//     and the other rows 2, 3 of each group of four (the row class is uniform
//     over the workgroup, so it stays compile-time);
//   * each thread loads its own column strip of RY + 2q rows (the y halo wraps
//     periodically) straight into registers and does the y pass there
//     (P = My x, S = Ky x); only P and S go through LDS, double-buffered, for
//     the x pass across element columns -- one barrier per plane;
//   * the x pass reads the neighbouring element columns (periodic wrap) and
//     produces g, h; the z pass is done element layer by element layer with
//     q+1 accumulators per point (element form), so only the element layer
//     below the chunk is recomputed;
//   * the next plane's loads are issued before the current plane is computed;
//   * the smoother step and the apply with its dot keep the centre rows of the
//     planes of the current element layer for the epilogue's x;
//   * node classes (i mod q) are compile-time in y and z and per thread in x,
//     so structurally zero taps are never issued;
//   * blocks are remapped so each XCD (blockIdx mod 8) sweeps a contiguous
//     range of tiles and shares the y halos in its own L2.
//
// k_apply_pt (levels with N <= 32, latency-bound): one thread per element
//   column of one row sums its (2q+1)^3 neighbourhood by sum factorization in
//   registers; the whole level sits in cache.  For q >= 2 the 2q+1 z rows of
//   the neighbourhood go to 2q+1 wavefronts and their partial sums meet in LDS.
//
// FP32 q = 4 on the matrix cores: the x and z passes of the column kernel are
//   v_mfma_f32_4x4x1_16b_f32 outer products.  Lane l's four result registers
//   hold sum_k A(lane 4 (l / 4) + v) B(lane l), v = 0 .. 3: each lane gives one
//   value of its own element column as B and the lanes of its group of four give
//   the weights of node class v as A, so one instruction adds one tap (x pass) or
//   one plane of the element layer (z pass) to all four classes or output planes
//   of every lane.  Only the vertex's taps into the left element (x) and the
//   shared top plane (z) stay on the vector unit.
//
// Epilogues fuse the residual (b - A x) and the Chebyshev-Jacobi step
// x + c1 (x - x_prev) + c2 D^-1 (b - A x) into the same pass.  From a zero
// guess the first two steps are one pass: the input values are b scaled by
// s0 D^-1 as they are loaded (x_1, one multiply in the kernel's precision),
// and the epilogue stores x_1 beside x_2.
#include <map>
#include <mutex>
#include <utility>

#include "gmg_kernels.h"

namespace gmg {
namespace {

typedef float mf4 __attribute__((ext_vector_type(4)));

// Instances with a matrix-core form of the column kernel (ApplyArgs::mfma).
template <typename T, int Q>
constexpr bool col_mfma_ok() {
  return sizeof(T) == 4 && Q == 4;
}

// one tap: d[v] += A(lane 4 (l / 4) + v) * B(lane l)
__device__ __forceinline__ mf4 mfma4(float a, float b, mf4 d) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, d, 0, 0, 0);
}

// the value of four by node class c = 0 .. 3
__device__ __forceinline__ float by_class(int c, float v0, float v1, float v2, float v3) {
  return c == 0 ? v0 : c == 1 ? v1 : c == 2 ? v2 : v3;
}

template <typename T, int Q>
struct alignas(sizeof(T) * Q) VecQ {
  T v[Q];
};

template <typename T, int Q>
struct KTab {
  T kr[Q][2 * Q + 1];
  T mr[Q][2 * Q + 1];
  T zk[Q + 1][Q + 1];
  T zm[Q + 1][Q + 1];
  T zkr[Q][2 * Q + 1];
  T zmr[Q][2 * Q + 1];
  T dinv[Q * Q * Q];
  T fz[Q * Q * Q];  // s0 D^-1 by node class (first steps from a zero guess)
};

constexpr int kEpiZero = static_cast<int>(Epi::ChebZero);
constexpr int kEpiDot = static_cast<int>(Epi::ApplyDot);
constexpr int kEpiResSums = static_cast<int>(Epi::ResidualSums);
constexpr int kEpiResNorms = static_cast<int>(Epi::ResidualNorms);
// epilogues that reduce two sums per block into a partials buffer
constexpr bool reduces(int epi) { return epi == kEpiDot || epi == kEpiResSums || epi == kEpiResNorms; }

// x_1 = s0 D^-1 b at one node of class cls
template <typename T, int Q>
__device__ __forceinline__ T x1_of(const KTab<T, Q>& tb, int cls, T b) {
  return tb.fz[cls] * b;
}

// Is offset o (in -Q..Q) a structural nonzero of the assembled 1D row of class c?
__host__ __device__ constexpr bool tap(int Q, int c, int o) {
  return c == 0 ? true : (o >= -c && o <= Q - c);
}

// Non-temporal q-wide store: the output of a plain apply is not read again by
// the kernel, and keeping it out of the L2 leaves room for the input halos
// (measured: 512^3 DoF applies about 6% faster, except FP64 q = 4, which is
// slower with it; the smoother steps, whose output is the next step's input,
// are slower with it and do not use it).
template <typename T, int Q>
__device__ __forceinline__ void store_nt(T* p, const VecQ<T, Q>& v) {
  if constexpr (Q == 1) {
    __builtin_nontemporal_store(v.v[0], p);
  } else {
    typedef T vt __attribute__((ext_vector_type(Q)));
    vt w;
#pragma unroll
    for (int c = 0; c < Q; ++c) w[c] = v.v[c];
    __builtin_nontemporal_store(w, reinterpret_cast<vt*>(p));
  }
}

// Fused epilogue on one q-wide output vector.  xc: the input values at idx when the caller
// still holds them in registers, else null and they are read again from memory.
template <typename T, int Q, int EPI>
__device__ __forceinline__ void emit(const KTab<T, Q>& tb, const size_t idx, const int cy, const int cz,
                                     const T (&ax)[Q], const T* __restrict__ x, T* out, const T* bvec,
                                     const T* xp, const T c1, const T c2, T* x1o, double (&dacc)[2],
                                     const VecQ<T, Q>* xc = nullptr) {
  using V = VecQ<T, Q>;
  V res;
  if constexpr (EPI == kEpiDot) {
    const V xv = xc ? *xc : *reinterpret_cast<const V*>(x + idx);
#pragma unroll
    for (int c = 0; c < Q; ++c) {
      res.v[c] = ax[c];
      dacc[0] = fma(static_cast<double>(xv.v[c]), static_cast<double>(ax[c]), dacc[0]);
      dacc[1] += static_cast<double>(ax[c]);
    }
    if constexpr (Q < 4 || sizeof(T) == 4) {
      store_nt<T, Q>(out + idx, res);
      return;
    }
  } else if constexpr (EPI == kEpiZero) {
    const V bv = *reinterpret_cast<const V*>(bvec + idx);
    V x1;
#pragma unroll
    for (int c = 0; c < Q; ++c) {
      const int cls = c + Q * (cy + Q * cz);
      x1.v[c] = x1_of(tb, cls, bv.v[c]);
      res.v[c] = x1.v[c] + c1 * (x1.v[c] - T(0)) + c2 * tb.dinv[cls] * (bv.v[c] - ax[c]);
    }
    *reinterpret_cast<V*>(x1o + idx) = x1;
  } else if constexpr (EPI == static_cast<int>(Epi::Apply)) {
#pragma unroll
    for (int c = 0; c < Q; ++c) res.v[c] = ax[c];
    if constexpr (Q < 4 || sizeof(T) == 4) {
      store_nt<T, Q>(out + idx, res);
      return;
    }
  } else if constexpr (EPI == kEpiResSums) {
    const V bv = *reinterpret_cast<const V*>(bvec + idx);
#pragma unroll
    for (int c = 0; c < Q; ++c) {
      res.v[c] = bv.v[c] - ax[c];
      dacc[0] = fma(static_cast<double>(res.v[c]), static_cast<double>(res.v[c]), dacc[0]);
      dacc[1] += static_cast<double>(res.v[c]);
    }
  } else if constexpr (EPI == kEpiResNorms) {
    // |b - A x|^2 and |b|^2 of this thread's outputs (the test of a learned cycle); no store
    const V bv = *reinterpret_cast<const V*>(bvec + idx);
#pragma unroll
    for (int c = 0; c < Q; ++c) {
      const T r = bv.v[c] - ax[c];
      dacc[0] = fma(static_cast<double>(r), static_cast<double>(r), dacc[0]);
      dacc[1] = fma(static_cast<double>(bv.v[c]), static_cast<double>(bv.v[c]), dacc[1]);
    }
    return;
  } else if constexpr (EPI == static_cast<int>(Epi::Residual)) {
    const V bv = *reinterpret_cast<const V*>(bvec + idx);
#pragma unroll
    for (int c = 0; c < Q; ++c) res.v[c] = bv.v[c] - ax[c];
  } else {
    const V bv = *reinterpret_cast<const V*>(bvec + idx);
    const V xv = xc ? *xc : *reinterpret_cast<const V*>(x + idx);
    V pv;
    if (c1 != T(0)) {
      if (xp != nullptr) {
        pv = *reinterpret_cast<const V*>(xp + idx);
      } else {
#pragma unroll
        for (int c = 0; c < Q; ++c) pv.v[c] = T(0);
      }
    } else {
#pragma unroll
      for (int c = 0; c < Q; ++c) pv.v[c] = xv.v[c];
    }
#pragma unroll
    for (int c = 0; c < Q; ++c) {
      const T dinv = tb.dinv[c + Q * (cy + Q * cz)];
      res.v[c] = xv.v[c] + c1 * (xv.v[c] - pv.v[c]) + c2 * dinv * (bv.v[c] - ax[c]);
    }
  }
  *reinterpret_cast<V*>(out + idx) = res;
}

template <int Q>
constexpr int col_bound() {
  return Q == 4 ? 256 : 512;
}

// Rows per thread of the column kernel: FP64 q = 4 and the FP64 q = 2 smoother
// steps (whose epilogue holds three more vectors) and reducing epilogues take two,
// or their element-layer accumulators would spill; the rest take four (measured on
// 256^3 DoFs: FP64 q = 2 smoother step 140 -> 117 us with two rows, the apply with
// its two sums 70 -> 49 us, the plain FP64 apply slower with two).  FP32 q = 2
// residuals and smoother steps take two as well: 110 instead of 174-190 VGPRs, four
// wavefronts per SIMD instead of two, which their extra input streams need to keep
// memory busy (512^3 DoFs: smoother step 550 -> 444 us, residual 434 -> 371 us; the
// plain apply is faster with four, 243 against 274 us).  So do the FP32 q = 4 ones:
// two wavefronts per SIMD instead of one (512^3 DoFs: smoother step 732 -> 495 us,
// residual 520 -> 378 us; the plain apply 309 us with four rows, 323 with two).
template <typename T, int Q, int EPI>
constexpr int col_rows() {
  if (sizeof(T) != 8)
    return ((Q == 2 || Q == 4) && (EPI == static_cast<int>(Epi::Residual) || EPI == static_cast<int>(Epi::Cheb) ||
                       EPI == static_cast<int>(Epi::ChebZero) || EPI == kEpiResNorms))
               ? 2
               : 4;
  if (Q == 4) return 2;
  if (Q == 2 && (EPI == static_cast<int>(Epi::Cheb) || EPI == static_cast<int>(Epi::ChebZero) ||
                 EPI == static_cast<int>(Epi::ApplyDot) || EPI == static_cast<int>(Epi::ResidualSums) ||
                 EPI == kEpiResNorms))
    return 2;
  return 4;
}

// --------------------------------------------------------------------------
// Streaming column kernel.
// Body of the column kernel for workgroups whose threads start at row class CY0.
template <typename T, int Q, int G, int EPI, int RY, int CY0, bool PRE, bool MFK>
__device__ __forceinline__ void col_body(const T* __restrict__ x, const KTab<T, Q>& tb, const int N, const int TZ,
                                         const int Y0, const int E0, T* out, const T* bvec, const T* xp,
                                         const T c1, const T c2, T* x1o, double (&dacc)[2]) {
  constexpr int TY = G * RY;
  constexpr int NR = RY + 2 * Q;
  constexpr bool kLatePrefetch = Q == 4;
  using V = VecQ<T, Q>;

  const int tx = threadIdx.x;
  const int ty = threadIdx.y;
  const int NX = N / Q;
  const int Nm = N - 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);  // [2 buffers][P,S][TY][N]
  const int buf_stride = 2 * TY * N;
  const size_t NN = static_cast<size_t>(N) * N;
  const int yrow0 = Y0 + 4 * ty + CY0;  // first output row of this thread

  // offsets (in elements) of the strip rows inside a plane, y wrapping periodically
  int roff[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) roff[r] = ((yrow0 - Q + r) & Nm) * N + Q * tx;

  V pre[NR];
  // cz: the plane's z class (p mod q), passed so that it stays a compile-time value where
  // the plane is chosen at run time
  auto load_cls = [&](V(&dst)[NR], int p, int cz) {
    const T* base = x + static_cast<size_t>(p & Nm) * NN;
#pragma unroll
    for (int r = 0; r < NR; ++r) dst[r] = *reinterpret_cast<const V*>(base + roff[r]);
    if constexpr (EPI == kEpiZero) {
      // strip row r has y class (CY0 + r) mod q, the plane z class cz
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int c = 0; c < Q; ++c) dst[r].v[c] = x1_of(tb, c + Q * ((CY0 + r) % Q + Q * cz), dst[r].v[c]);
    }
  };
  auto load_to = [&](V(&dst)[NR], int p) { load_cls(dst, p, p & (Q - 1)); };
  auto load_plane = [&](int p) { load_to(pre, p); };
  // the next plane, or past the chunk's end plane p + 1 - q (same z class, loaded q - 1
  // planes ago, still in cache; its values are not used)
  auto prefetch_next = [&](int p, bool prefetch) { load_cls(pre, prefetch ? p + 1 : p + 1 - Q, (p + 1) & (Q - 1)); };

  const int txl = (tx - 1) & (NX - 1);
  const int txr = (tx + 1) & (NX - 1);
  T g[RY][Q], h[RY][Q];
  int parity = 0;
  // epilogues that need x at the output point keep the RY centre rows of the planes of the
  // current element layer (slot b: plane E q + b) instead of reading them again from memory
  // (512^3 DoFs, FP32 q = 2 smoother step: 444 -> 421 us)
  constexpr bool kKeep = Q <= 2 && (EPI == static_cast<int>(Epi::Cheb) || EPI == kEpiDot);
  V xcen[kKeep ? Q + 1 : 1][RY];
  auto keep = [&](const V (&xv)[NR], int slot) {
    if constexpr (kKeep) {
#pragma unroll
      for (int i = 0; i < RY; ++i) xcen[slot][i] = xv[Q + i];
    }
  };

  // y pass in registers: P = My x and S = Ky x of the RY output rows into LDS
  auto ypass = [&](const V (&xv)[NR], T* ps, T* ss) {
#pragma unroll
    for (int i = 0; i < RY; ++i) {
      const int ci = (CY0 + i) % Q;
      V pv, sv;
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        pv.v[c] = T(0);
        sv.v[c] = T(0);
      }
#pragma unroll
      for (int o = -Q; o <= Q; ++o) {
        if (!tap(Q, ci, o)) continue;
        const T m = tb.mr[ci][o + Q];
        const T k = tb.kr[ci][o + Q];
#pragma unroll
        for (int c = 0; c < Q; ++c) {
          pv.v[c] = fma(m, xv[i + Q + o].v[c], pv.v[c]);
          sv.v[c] = fma(k, xv[i + Q + o].v[c], sv.v[c]);
        }
      }
      *reinterpret_cast<V*>(ps + (ty * RY + i) * N + Q * tx) = pv;
      *reinterpret_cast<V*>(ss + (ty * RY + i) * N + Q * tx) = sv;
    }
  };

  // matrix-core form (FP32 q = 4): per-lane A operands, row (tx & 3) of each weight
  // table.  x pass: window tap Q + j of node class c is table column Q + j - c; z pass:
  // output plane c from plane j of the element layer.
  constexpr bool MF = MFK && col_mfma_ok<T, Q>();
  constexpr int NMF = MF ? Q + 1 : 1;
  float xkA[NMF], xmA[NMF], zkA[NMF], zmA[NMF];
  if constexpr (MF) {
    const int cl = tx & 3;
#pragma unroll
    for (int j = 0; j <= Q; ++j) {
      xkA[j] = by_class(cl, tb.kr[0][Q + j], tb.kr[1][Q + j - 1], tb.kr[2][Q + j - 2], tb.kr[3][Q + j - 3]);
      xmA[j] = by_class(cl, tb.mr[0][Q + j], tb.mr[1][Q + j - 1], tb.mr[2][Q + j - 2], tb.mr[3][Q + j - 3]);
      zkA[j] = by_class(cl, tb.zk[0][j], tb.zk[1][j], tb.zk[2][j], tb.zk[3][j]);
      zmA[j] = by_class(cl, tb.zm[0][j], tb.zm[1][j], tb.zm[2][j], tb.zm[3][j]);
    }
  }

  // x pass across element columns, after the y pass of this plane went to LDS
  auto xpass = [&]() {
    T* ps = lds + parity * buf_stride;
    T* ss = ps + TY * N;
    if constexpr (MF) {
#pragma unroll
      for (int i = 0; i < RY; ++i) {
        const int row = (ty * RY + i) * N;
        const V a = *reinterpret_cast<const V*>(ps + row + Q * txl);
        const V b = *reinterpret_cast<const V*>(ps + row + Q * tx);
        const T c = ps[row + Q * txr];
        const V d = *reinterpret_cast<const V*>(ss + row + Q * txl);
        const V e = *reinterpret_cast<const V*>(ss + row + Q * tx);
        const T f = ss[row + Q * txr];
        // own element column and the right vertex: every class has these taps
        mf4 gv = {0.f, 0.f, 0.f, 0.f}, hv = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          gv = mfma4(xkA[j], b.v[j], gv);
          gv = mfma4(xmA[j], e.v[j], gv);
          hv = mfma4(xmA[j], b.v[j], hv);
        }
        gv = mfma4(xkA[Q], c, gv);
        gv = mfma4(xmA[Q], f, gv);
        hv = mfma4(xmA[Q], c, hv);
        // the vertex (class 0) also reaches into the left element column (offsets -q .. -1)
        T g0 = gv[0], h0 = hv[0];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          g0 = fma(tb.kr[0][k], a.v[k], g0);
          g0 = fma(tb.mr[0][k], d.v[k], g0);
          h0 = fma(tb.mr[0][k], a.v[k], h0);
        }
        g[i][0] = g0;
        h[i][0] = h0;
#pragma unroll
        for (int cc = 1; cc < Q; ++cc) {
          g[i][cc] = gv[cc];
          h[i][cc] = hv[cc];
        }
      }
      parity ^= 1;
      return;
    }
#pragma unroll
    for (int i = 0; i < RY; ++i) {
      const int row = (ty * RY + i) * N;
      T pw[2 * Q + 1], sw[2 * Q + 1];
      {
        const V a = *reinterpret_cast<const V*>(ps + row + Q * txl);
        const V b = *reinterpret_cast<const V*>(ps + row + Q * tx);
        const T c = ps[row + Q * txr];
        const V d = *reinterpret_cast<const V*>(ss + row + Q * txl);
        const V e = *reinterpret_cast<const V*>(ss + row + Q * tx);
        const T f = ss[row + Q * txr];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          pw[k] = a.v[k];
          pw[Q + k] = b.v[k];
          sw[k] = d.v[k];
          sw[Q + k] = e.v[k];
        }
        pw[2 * Q] = c;
        sw[2 * Q] = f;
      }
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        T gg = T(0), hh = T(0);
#pragma unroll
        for (int o = -Q; o <= Q; ++o) {
          if (!tap(Q, c, o)) continue;
          const T pv = pw[Q + c + o];
          const T sv = sw[Q + c + o];
          gg = fma(tb.kr[c][o + Q], pv, gg);
          gg = fma(tb.mr[c][o + Q], sv, gg);
          hh = fma(tb.mr[c][o + Q], pv, hh);
        }
        g[i][c] = gg;
        h[i][c] = hh;
      }
    }
    parity ^= 1;
  };

  // The next plane's loads go out on every plane, with no branch around them (past the
  // chunk's last plane q <= 2 reads plane p + 1 - q again, in cache, and q = 4 the next
  // chunk's first plane; the values are not used): behind a branch the compiler waited on
  // the loads right after issuing them -- q = 4 moved the next y pass into the branch,
  // q <= 2 copied the loaded rows into the strip registers at the join -- so no load
  // overlapped the compute (512^3 DoFs: q = 4 FP32 apply 335 -> 309 us, FP64 smoother step
  // 1086 -> 907 us; q = 2 FP32 smoother step 3.5 % and residual 5 % faster, the C4 FP32
  // solve 39.3 -> 38.4 ms).
  auto compute_gh = [&](int p, bool prefetch, int slot) {
    T* ps = lds + parity * buf_stride;
    T* ss = ps + TY * N;
    if constexpr (kLatePrefetch) {
      // the next plane's loads go out once the y pass has consumed this one: one strip
      // of registers instead of two (q = 4 would spill), the loads still overlap the
      // x and z passes
      ypass(pre, ps, ss);
      keep(pre, slot);
      // q = 4 takes the next plane even past the chunk's end (a plane of the next chunk, in
      // bounds through the periodic wrap): the chosen address costs the zero-start step a
      // spill at its 256-register limit
      load_plane(p + 1);
    } else {
      V xv[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) xv[r] = pre[r];
      prefetch_next(p, prefetch);
      ypass(xv, ps, ss);
      keep(xv, slot);
    }
    __syncthreads();
    xpass();
  };

  T acc[RY][Q][Q + 1];
  if constexpr (PRE) {
    // a one-layer chunk (TZ = 1): the 2q+1 planes (E0-1) q .. (E0+1) q are loaded at
    // once, so the block waits for memory once instead of once per plane
    V allp[2 * Q + 1][NR];
#pragma unroll
    for (int k = 0; k <= 2 * Q; ++k) load_to(allp[k], (E0 - 1) * Q + k);
    auto gh_of = [&](int k) {
      T* ps = lds + parity * buf_stride;
      ypass(allp[k], ps, ps + TY * N);
      __syncthreads();
      xpass();
    };
    gh_of(0);
#pragma unroll
    for (int i = 0; i < RY; ++i)
#pragma unroll
      for (int c = 0; c < Q; ++c)
#pragma unroll
        for (int a = 0; a <= Q; ++a) acc[i][c][a] = tb.zm[a][0] * g[i][c] + tb.zk[a][0] * h[i][c];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
#pragma unroll
      for (int b = 1; b <= Q; ++b) {
        gh_of(e * Q + b);
#pragma unroll
        for (int i = 0; i < RY; ++i)
#pragma unroll
          for (int c = 0; c < Q; ++c)
#pragma unroll
            for (int a = 0; a <= Q; ++a)
              acc[i][c][a] = fma(tb.zm[a][b], g[i][c], fma(tb.zk[a][b], h[i][c], acc[i][c][a]));
      }
      if (e == 1) {
#pragma unroll
        for (int a = 0; a < Q; ++a) {
          const size_t zoff = static_cast<size_t>(E0 * Q + a) * NN;
#pragma unroll
          for (int i = 0; i < RY; ++i) {
            T ax[Q];
#pragma unroll
            for (int c = 0; c < Q; ++c) ax[c] = acc[i][c][a];
            const size_t idx = zoff + static_cast<size_t>(yrow0 + i) * N + Q * tx;
            emit<T, Q, EPI>(tb, idx, (CY0 + i) % Q, a, ax, x, out, bvec, xp, c1, c2, x1o, dacc,
                            kKeep ? &allp[Q + a][Q + i] : nullptr);
          }
        }
      } else {
        // carry the shared vertex plane into element layer E0
#pragma unroll
        for (int i = 0; i < RY; ++i)
#pragma unroll
          for (int c = 0; c < Q; ++c) {
            const T top = acc[i][c][Q];
            acc[i][c][0] = top + tb.zm[0][0] * g[i][c] + tb.zk[0][0] * h[i][c];
#pragma unroll
            for (int a = 1; a <= Q; ++a) acc[i][c][a] = tb.zm[a][0] * g[i][c] + tb.zk[a][0] * h[i][c];
          }
      }
    }
    return;
  }
  const int zlast = (E0 + TZ) * Q;
  if constexpr (MF) {
    // z pass in element form on the matrix cores: four of the q + 1 accumulators of a
    // point in one mf4 (output planes 0 .. 3 of the element layer), the shared top plane
    // (slot q) on the vector unit.  Plane 0 of a layer starts them (with carry adding the
    // top plane the layer below left), each further plane b adds its two terms.
    mf4 acc4[RY][Q];
    T top[RY][Q];
    auto z_first = [&](bool carry) {
#pragma unroll
      for (int i = 0; i < RY; ++i)
#pragma unroll
        for (int c = 0; c < Q; ++c) {
          mf4 t = mfma4(zmA[0], g[i][c], mf4{0.f, 0.f, 0.f, 0.f});
          t = mfma4(zkA[0], h[i][c], t);
          if (carry) t[0] += top[i][c];
          acc4[i][c] = t;
          top[i][c] = tb.zm[Q][0] * g[i][c] + tb.zk[Q][0] * h[i][c];
        }
    };
    load_plane((E0 - 1) * Q);
    compute_gh((E0 - 1) * Q, true, 0);
    z_first(false);
    for (int E = E0 - 1; E < E0 + TZ; ++E) {
#pragma unroll
      for (int b = 1; b <= Q; ++b) {
        const int p = E * Q + b;
        compute_gh(p, p < zlast, b);
#pragma unroll
        for (int i = 0; i < RY; ++i)
#pragma unroll
          for (int c = 0; c < Q; ++c) {
            acc4[i][c] = mfma4(zmA[b], g[i][c], mfma4(zkA[b], h[i][c], acc4[i][c]));
            top[i][c] = fma(tb.zm[Q][b], g[i][c], fma(tb.zk[Q][b], h[i][c], top[i][c]));
          }
      }
      if (E >= E0) {
#pragma unroll
        for (int a = 0; a < Q; ++a) {
          const size_t zoff = static_cast<size_t>(E * Q + a) * NN;
#pragma unroll
          for (int i = 0; i < RY; ++i) {
            T ax[Q];
#pragma unroll
            for (int c = 0; c < Q; ++c) ax[c] = acc4[i][c][a];
            const size_t idx = zoff + static_cast<size_t>(yrow0 + i) * N + Q * tx;
            emit<T, Q, EPI>(tb, idx, (CY0 + i) % Q, a, ax, x, out, bvec, xp, c1, c2, x1o, dacc, nullptr);
          }
        }
      }
      z_first(true);  // carry the shared vertex plane into the next element layer
    }
    return;
  }

  load_plane((E0 - 1) * Q);
  compute_gh((E0 - 1) * Q, true, 0);
#pragma unroll
  for (int i = 0; i < RY; ++i)
#pragma unroll
    for (int c = 0; c < Q; ++c)
#pragma unroll
      for (int a = 0; a <= Q; ++a) acc[i][c][a] = tb.zm[a][0] * g[i][c] + tb.zk[a][0] * h[i][c];

  for (int E = E0 - 1; E < E0 + TZ; ++E) {
#pragma unroll
    for (int b = 1; b <= Q; ++b) {
      const int p = E * Q + b;
      compute_gh(p, p < zlast, b);
#pragma unroll
      for (int i = 0; i < RY; ++i)
#pragma unroll
        for (int c = 0; c < Q; ++c)
#pragma unroll
          for (int a = 0; a <= Q; ++a)
            acc[i][c][a] = fma(tb.zm[a][b], g[i][c], fma(tb.zk[a][b], h[i][c], acc[i][c][a]));
    }
    if (E >= E0) {
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        const size_t zoff = static_cast<size_t>(E * Q + a) * NN;
#pragma unroll
        for (int i = 0; i < RY; ++i) {
          T ax[Q];
#pragma unroll
          for (int c = 0; c < Q; ++c) ax[c] = acc[i][c][a];
          const size_t idx = zoff + static_cast<size_t>(yrow0 + i) * N + Q * tx;
          emit<T, Q, EPI>(tb, idx, (CY0 + i) % Q, a, ax, x, out, bvec, xp, c1, c2, x1o, dacc,
                          kKeep ? &xcen[a][i] : nullptr);
        }
      }
    }
    if constexpr (kKeep) {  // plane (E + 1) q is slot 0 of the next layer
#pragma unroll
      for (int i = 0; i < RY; ++i) xcen[0][i] = xcen[Q][i];
    }
    // carry the shared vertex plane into the next element layer
#pragma unroll
    for (int i = 0; i < RY; ++i)
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        const T top = acc[i][c][Q];
        acc[i][c][0] = top + tb.zm[0][0] * g[i][c] + tb.zk[0][0] * h[i][c];
#pragma unroll
        for (int a = 1; a <= Q; ++a) acc[i][c][a] = tb.zm[a][0] * g[i][c] + tb.zk[a][0] * h[i][c];
      }
  }
}

// Wavefronts per SIMD the compiler is held to: two for the two-row FP32 q = 4 instances
// (left alone, the zero-guess smoother step took 266 registers and so one wavefront; held
// to two it needs 240 and spills nothing), the compiler's own choice elsewhere.
template <typename T, int Q, int EPI>
constexpr int col_min_waves() {
  return (sizeof(T) == 4 && Q == 4 && col_rows<T, Q, EPI>() == 2) ? 2 : 1;
}

template <typename T, int Q, int G, int EPI, bool PRE = false, bool MF = false>
__global__ void __launch_bounds__(col_bound<Q>()) __attribute__((amdgpu_waves_per_eu(col_min_waves<T, Q, EPI>())))
k_apply_col(const T* __restrict__ x, const KTab<T, Q> tb,
                                                              const int N, const int TZ, const int ntiles_y,
                                                              T* out, const T* bvec, const T* xp, const T c1,
                                                              const T c2, T* x1o, double* part) {
  constexpr int RY = col_rows<T, Q, EPI>();
  constexpr int SPLIT = 4 / RY;  // workgroups per tile
  const int nblocks = gridDim.x;
  int b = blockIdx.x;
  if ((nblocks & 7) == 0) b = (blockIdx.x & 7) * (nblocks >> 3) + (blockIdx.x >> 3);
  const int tile = b / SPLIT;
  const int Y0 = (tile % ntiles_y) * 4 * G;
  const int E0 = (tile / ntiles_y) * TZ;
  double dacc[2] = {0.0, 0.0};
  if constexpr (SPLIT == 1) {
    col_body<T, Q, G, EPI, RY, 0, PRE, MF>(x, tb, N, TZ, Y0, E0, out, bvec, xp, c1, c2, x1o, dacc);
  } else {
    if (b % SPLIT == 0) col_body<T, Q, G, EPI, RY, 0, PRE, MF>(x, tb, N, TZ, Y0, E0, out, bvec, xp, c1, c2, x1o, dacc);
    else col_body<T, Q, G, EPI, RY, 2, PRE, MF>(x, tb, N, TZ, Y0, E0, out, bvec, xp, c1, c2, x1o, dacc);
  }
  if constexpr (reduces(EPI)) {
    // block partials in a fixed order: wavefront shuffles, then the wavefronts in turn
    __shared__ double red[2][col_bound<Q>() / 64];
#pragma unroll
    for (int k = 0; k < 2; ++k)
      for (int off = 32; off > 0; off >>= 1) dacc[k] += __shfl_down(dacc[k], off, 64);
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const int nw = (blockDim.x * blockDim.y) >> 6;
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = dacc[0];
      red[1][tid >> 6] = dacc[1];
    }
    __syncthreads();
    if (tid == 0) {
      double s0 = 0.0, s1 = 0.0;
      for (int w = 0; w < nw; ++w) {
        s0 += red[0][w];
        s1 += red[1][w];
      }
      part[blockIdx.x] = s0;
      part[nblocks + blockIdx.x] = s1;
    }
  }
}

// --------------------------------------------------------------------------
// Point kernel for small levels: thread = one element column (q nodes) of one
// row.  With KZ > 1 (q >= 2) the 2q+1 z rows of the neighbourhood are split over
// the KZ = 2q+1 wavefronts of a block (one z row each, so the row loads of a
// thread are one round of latency instead of 2q+1, and a 32^3-node level has
// 2q+1 times the threads), and the partial sums are added in LDS in a fixed order
// (measured for q = 2 on 32^3 nodes: smoother step 6.3 -> 4.9 us).
template <int KZ>
constexpr int pt_threads() {
  return KZ == 1 ? 128 : 64 * KZ;
}

template <typename T, int Q, int EPI, int KZ>
__global__ void __launch_bounds__(pt_threads<KZ>()) k_apply_pt(const T* __restrict__ x, const KTab<T, Q> tb,
                                                               const int N, T* out, const T* bvec, const T* xp,
                                                               const T c1, const T c2, T* x1o) {
  constexpr int kCols = KZ == 1 ? 128 : 64;  // element columns per block (blockDim.x)
  const int NX = N / Q;
  const int64_t total = static_cast<int64_t>(NX) * N * N;
  const int64_t t = blockIdx.x * static_cast<int64_t>(kCols) + threadIdx.x;
  const bool live = t < total;
  const int64_t tt = live ? t : 0;
  const int Nm = N - 1;
  const int tx = static_cast<int>(tt % NX);
  const int yy = static_cast<int>((tt / NX) % N);
  const int zz = static_cast<int>(tt / (static_cast<int64_t>(NX) * N));
  const int cy = yy % Q;
  const int cz = zz % Q;
  // sum over the (dz, dy) rows of the neighbourhood of
  //   (Kx row . x) My Zm + (Mx row . x) (Ky Zm + My Zk)
  // with (Zm, Zk) = (Mz, Kz) for the stiffness and (0, Mz) for the mass
  T ax[Q];
#pragma unroll
  for (int c = 0; c < Q; ++c) ax[c] = T(0);
  auto zrow = [&](const int dz) {
    const T mz = tb.zmr[cz][dz + Q], kz = tb.zkr[cz][dz + Q];
    const int zr = (zz + dz) & Nm;
#pragma unroll
    for (int dy = -Q; dy <= Q; ++dy) {
      const T my = tb.mr[cy][dy + Q], ky = tb.kr[cy][dy + Q];
      const int yr = (yy + dy) & Nm;
      const T* row = x + (static_cast<size_t>(zr) * N + yr) * N;
      const T wk = my * mz;            // weight of the Kx row product
      const T wm = ky * mz + my * kz;  // weight of the Mx row product
      T xr[2 * Q + 1];
#pragma unroll
      for (int k = 0; k <= 2 * Q; ++k) xr[k] = row[(Q * tx - Q + k + N) & Nm];
      if constexpr (EPI == kEpiZero) {
        // node (Q tx - Q + k) has x class k mod q
        const int base = Q * ((yr & (Q - 1)) + Q * (zr & (Q - 1)));
#pragma unroll
        for (int k = 0; k <= 2 * Q; ++k) xr[k] = x1_of(tb, base + k % Q, xr[k]);
      }
#pragma unroll
      for (int c = 0; c < Q; ++c) {
        T rk = T(0), rm = T(0);
#pragma unroll
        for (int o = -Q; o <= Q; ++o) {
          if (!tap(Q, c, o)) continue;
          rk = fma(tb.kr[c][o + Q], xr[Q + c + o], rk);
          rm = fma(tb.mr[c][o + Q], xr[Q + c + o], rm);
        }
        ax[c] = fma(wk, rk, fma(wm, rm, ax[c]));
      }
    }
  };
  if constexpr (KZ == 1) {
    if (!live) return;
    // unrolled so that all (2q+1)^2 row loads can be in flight at once;
    // taps outside a row's band carry zero weights
#pragma unroll
    for (int dz = -Q; dz <= Q; ++dz) zrow(dz);
  } else {
    static_assert(KZ == 2 * Q + 1, "one z row per wavefront");
    __shared__ T part[KZ][kCols][Q];
    if (live) zrow(static_cast<int>(threadIdx.y) - Q);
#pragma unroll
    for (int c = 0; c < Q; ++c) part[threadIdx.y][threadIdx.x][c] = ax[c];
    __syncthreads();
    if (!live || threadIdx.y != 0) return;
#pragma unroll
    for (int c = 0; c < Q; ++c) {
      T s = part[0][threadIdx.x][c];
#pragma unroll
      for (int g = 1; g < KZ; ++g) s += part[g][threadIdx.x][c];
      ax[c] = s;
    }
  }
  const size_t idx = (static_cast<size_t>(zz) * N + yy) * N + Q * tx;
  double dacc[2] = {0.0, 0.0};
  emit<T, Q, EPI>(tb, idx, cy, cz, ax, x, out, bvec, xp, c1, c2, x1o, dacc);
}

template <typename T, int Q>
KTab<T, Q> make_ktab(const OpTab& t, double s0) {
  KTab<T, Q> k{};
  for (int c = 0; c < Q; ++c)
    for (int o = 0; o < 2 * Q + 1; ++o) {
      k.kr[c][o] = static_cast<T>(t.krow[c][o]);
      k.mr[c][o] = static_cast<T>(t.mrow[c][o]);
      k.zkr[c][o] = static_cast<T>(t.zkrow[c][o]);
      k.zmr[c][o] = static_cast<T>(t.zmrow[c][o]);
    }
  for (int a = 0; a <= Q; ++a)
    for (int b = 0; b <= Q; ++b) {
      k.zk[a][b] = static_cast<T>(t.zk[a][b]);
      k.zm[a][b] = static_cast<T>(t.zm[a][b]);
    }
  for (int i = 0; i < Q * Q * Q; ++i) {
    k.dinv[i] = static_cast<T>(t.dinv[i]);
    k.fz[i] = static_cast<T>(s0 * t.dinv[i]);
  }
  return k;
}

// Launch shape of the column kernel on one level.
struct ColShape {
  int G, TZ, ntiles_y, nblocks, split;
  size_t lds;
};

// Rows per block and LDS of the column kernel on one level (the z chunk TZ is
// chosen at launch, from the kernel's occupancy).
inline ColShape col_shape(int N, int Q, size_t elem, int RY) {
  ColShape s{};
  const int nx = N / Q;
  s.split = 4 / RY;
  int G = 1;
  while (G < 4 && G * nx < 64 && 8 * G <= N) G *= 2;  // at least one full wavefront per block
  s.G = G;
  s.ntiles_y = N / (4 * G);
  s.lds = static_cast<size_t>(2 * 2 * RY * G) * N * elem;
  return s;
}

// Blocks of one column-kernel instance that the device holds at once: blocks per
// CU from the occupancy API (registers, LDS, block size) times the CU count.
// Cached per device and LDS size; the context primes it at setup, so no query
// runs while a launch sequence is being captured into a graph.
template <typename T, int Q, int G, int EPI, bool MF = false>
int resident_blocks(int threads, size_t lds) {
  static std::mutex mu;
  static std::map<std::pair<int, size_t>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_pair(dev, lds);
  const auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  const void* fn = reinterpret_cast<const void*>(&k_apply_col<T, Q, G, EPI, false, MF>);
  if (lds > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
  (void)hipGetLastError();
  return cache[key] = per_cu * cus;
}

// z chunk (element layers per block): each block streams its TZ layers plus one
// recomputed layer, and blocks run in rounds of `resident`; minimise
// rounds x (TZ + 1), preferring the larger chunk on ties.
inline int pick_tz(int n, int64_t tiles, int64_t resident) {
  int best = n;
  int64_t best_cost = -1;
  for (int TZ = n; TZ >= 1; TZ >>= 1) {
    const int64_t blocks = tiles * (n / TZ);
    const int64_t cost = (blocks + resident - 1) / resident * (TZ + 1);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = TZ;
    }
  }
  return best;
}

// the preloading variant: FP32 q <= 2 (2q+1 strips of registers), the plain epilogues
template <typename T, int Q, int EPI>
constexpr bool pre_ok() {
  return sizeof(T) == 4 && Q <= 2 && !reduces(EPI);
}

template <typename T, int Q, int G, int EPI, bool MF = false>
hipError_t launch_col(const KTab<T, Q>& kt, const ApplyArgs& a, ColShape sh, hipStream_t s) {
  if constexpr (col_mfma_ok<T, Q>() && !MF) {
    if (a.mfma) return launch_col<T, Q, G, EPI, true>(kt, a, sh, s);
  }
  const int threads = (a.N / Q) * G;
  const int64_t tiles = static_cast<int64_t>(sh.ntiles_y) * sh.split;
  sh.TZ = pick_tz(a.n, tiles, resident_blocks<T, Q, G, EPI, MF>(threads, sh.lds));
  sh.nblocks = static_cast<int>(tiles * (a.n / sh.TZ));
  if constexpr (reduces(EPI)) {
    if (a.part == nullptr || a.sc == nullptr || 2 * static_cast<int64_t>(sh.nblocks) > a.part_cap)
      return hipErrorInvalidValue;
  }
  if (sh.lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_apply_col<T, Q, G, EPI, false, MF>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(sh.lds));
    if (e != hipSuccess) return e;
  }
  if constexpr (pre_ok<T, Q, EPI>()) {
    if (sh.TZ == 1) {  // one element layer per block: all its planes loaded at once
      hipLaunchKernelGGL((k_apply_col<T, Q, G, EPI, true>), dim3(sh.nblocks), dim3(a.N / Q, G), sh.lds, s,
                         static_cast<const T*>(a.x), kt, a.N, sh.TZ, sh.ntiles_y, static_cast<T*>(a.out),
                         static_cast<const T*>(a.b), static_cast<const T*>(a.xp), static_cast<T>(a.c1),
                         static_cast<T>(a.c2), static_cast<T*>(a.x1), a.part);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_apply_col<T, Q, G, EPI, false, MF>), dim3(sh.nblocks), dim3(a.N / Q, G), sh.lds, s,
                     static_cast<const T*>(a.x), kt, a.N, sh.TZ, sh.ntiles_y, static_cast<T*>(a.out),
                     static_cast<const T*>(a.b), static_cast<const T*>(a.xp), static_cast<T>(a.c1),
                     static_cast<T>(a.c2), static_cast<T*>(a.x1), a.part);
  if constexpr (reduces(EPI)) {
    // the second run first: folding the first run writes into the second's place
    const int64_t nb = sh.nblocks;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_sum_partials(a.part + nb, nb, a.part_cap - nb, a.sc + a.d1, s);
    if (e != hipSuccess) return e;
    return launch_sum_partials(a.part, nb, a.part_cap, a.sc + a.d0, s);
  }
  return hipGetLastError();
}

template <typename T, int Q, int EPI>
hipError_t launch_te(const OpTab& tab, const ApplyArgs& a, hipStream_t s) {
  const KTab<T, Q> kt = make_ktab<T, Q>(tab, a.s0);
  if constexpr (reduces(EPI)) {
    if (a.N <= 32) return hipErrorInvalidValue;  // column kernel only
  } else if (a.N <= 32) {
    constexpr int KZ = Q >= 2 ? 2 * Q + 1 : 1;
    constexpr int cols = KZ == 1 ? 128 : 64;
    const int64_t total = static_cast<int64_t>(a.N / Q) * a.N * a.N;
    hipLaunchKernelGGL((k_apply_pt<T, Q, EPI, KZ>), dim3(static_cast<unsigned>((total + cols - 1) / cols)),
                       dim3(cols, KZ), 0, s, static_cast<const T*>(a.x), kt, a.N, static_cast<T*>(a.out),
                       static_cast<const T*>(a.b), static_cast<const T*>(a.xp), static_cast<T>(a.c1),
                       static_cast<T>(a.c2), static_cast<T*>(a.x1));
    return hipGetLastError();
  }
  const ColShape sh = col_shape(a.N, Q, sizeof(T), col_rows<T, Q, EPI>());
  if ((a.N / Q) * sh.G > col_bound<Q>()) return hipErrorInvalidConfiguration;
  switch (sh.G) {
    case 1: return launch_col<T, Q, 1, EPI>(kt, a, sh, s);
    case 2: return launch_col<T, Q, 2, EPI>(kt, a, sh, s);
    case 4: return launch_col<T, Q, 4, EPI>(kt, a, sh, s);
  }
  return hipErrorInvalidConfiguration;
}

template <typename T, int Q, int EPI, bool MF>
int resident_any(int G, int threads, size_t lds) {
  switch (G) {
    case 1: return resident_blocks<T, Q, 1, EPI, MF>(threads, lds);
    case 2: return resident_blocks<T, Q, 2, EPI, MF>(threads, lds);
    case 4: return resident_blocks<T, Q, 4, EPI, MF>(threads, lds);
  }
  return 1;
}

template <typename T, int Q, int EPI>
void prime_te(int N) {
  if (N <= 32) return;
  const ColShape sh = col_shape(N, Q, sizeof(T), col_rows<T, Q, EPI>());
  const int threads = (N / Q) * sh.G;
  resident_any<T, Q, EPI, false>(sh.G, threads, sh.lds);
  if constexpr (col_mfma_ok<T, Q>()) resident_any<T, Q, EPI, true>(sh.G, threads, sh.lds);
}

// The shape launch_te takes for one instance (a query for tests and tracing).
template <typename T, int Q, int EPI>
ApplyShape shape_te(int N, int n, bool mfma) {
  ApplyShape out{};
  if (N <= 32) {
    out.kernel = 0;
    constexpr int KZ = Q >= 2 ? 2 * Q + 1 : 1;
    constexpr int cols = KZ == 1 ? 128 : 64;
    out.G = 1;
    out.TZ = 0;
    out.nblocks = static_cast<int>((static_cast<int64_t>(N / Q) * N * N + cols - 1) / cols);
    return out;
  }
  ColShape sh = col_shape(N, Q, sizeof(T), col_rows<T, Q, EPI>());
  const int threads = (N / Q) * sh.G;
  bool mf = false;
  if constexpr (col_mfma_ok<T, Q>()) mf = mfma;
  const int resident = mf ? resident_any<T, Q, EPI, col_mfma_ok<T, Q>()>(sh.G, threads, sh.lds)
                          : resident_any<T, Q, EPI, false>(sh.G, threads, sh.lds);
  const int64_t tiles = static_cast<int64_t>(sh.ntiles_y) * sh.split;
  out.TZ = pick_tz(n, tiles, resident);
  out.G = sh.G;
  out.nblocks = static_cast<int>(tiles * (n / out.TZ));
  out.kernel = (pre_ok<T, Q, EPI>() && out.TZ == 1) ? 2 : mf ? 3 : 1;
  return out;
}

template <typename T, int Q>
ApplyShape shape_tq(Epi epi, int N, int n, bool mfma) {
  switch (epi) {
    case Epi::Apply: return shape_te<T, Q, 0>(N, n, mfma);
    case Epi::Residual: return shape_te<T, Q, 1>(N, n, mfma);
    case Epi::Cheb: return shape_te<T, Q, 2>(N, n, mfma);
    case Epi::ChebZero: return shape_te<T, Q, kEpiZero>(N, n, mfma);
    case Epi::ApplyDot:
      if constexpr (sizeof(T) == 8) return shape_te<T, Q, kEpiDot>(N, n, mfma);
      break;
    case Epi::ResidualSums:
      if constexpr (sizeof(T) == 8) return shape_te<T, Q, kEpiResSums>(N, n, mfma);
      break;
    case Epi::ResidualNorms: return shape_te<T, Q, kEpiResNorms>(N, n, mfma);
  }
  return ApplyShape{-1, 0, 0, 0};
}

template <typename T, int Q>
void prime_tq(int N) {
  prime_te<T, Q, 0>(N);
  prime_te<T, Q, 1>(N);
  prime_te<T, Q, 2>(N);
  prime_te<T, Q, kEpiZero>(N);
  prime_te<T, Q, kEpiResNorms>(N);
  if constexpr (sizeof(T) == 8) {
    prime_te<T, Q, kEpiDot>(N);
    prime_te<T, Q, kEpiResSums>(N);
  }
}

template <typename T, int Q>
hipError_t launch_tq(const OpTab& tab, const ApplyArgs& a, hipStream_t s) {
  switch (a.epi) {
    case Epi::Apply: return launch_te<T, Q, 0>(tab, a, s);
    case Epi::Residual: return launch_te<T, Q, 1>(tab, a, s);
    case Epi::Cheb: return launch_te<T, Q, 2>(tab, a, s);
    case Epi::ChebZero:
      if (a.x1 == nullptr || a.x != a.b) return hipErrorInvalidValue;
      return launch_te<T, Q, kEpiZero>(tab, a, s);
    case Epi::ApplyDot:
      if constexpr (sizeof(T) == 8) return launch_te<T, Q, kEpiDot>(tab, a, s);
      return hipErrorInvalidValue;
    case Epi::ResidualSums:
      if constexpr (sizeof(T) == 8) return launch_te<T, Q, kEpiResSums>(tab, a, s);
      return hipErrorInvalidValue;
    case Epi::ResidualNorms: return launch_te<T, Q, kEpiResNorms>(tab, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

int apply_max_elements_x(int q) { return q == 4 ? 256 : 512; }

void prime_apply_shapes(int q, int N) {
  switch (q) {
    case 1: prime_tq<float, 1>(N); prime_tq<double, 1>(N); break;
    case 2: prime_tq<float, 2>(N); prime_tq<double, 2>(N); break;
    case 4: prime_tq<float, 4>(N); prime_tq<double, 4>(N); break;
  }
}

ApplyShape apply_shape(int q, bool fp32, Epi epi, int N, int n, bool mfma) {
  if (N != q * n || N < 4 || (N & (N - 1)) != 0 || n > apply_max_elements_x(q)) return ApplyShape{-1, 0, 0, 0};
  switch (q) {
    case 1: return fp32 ? shape_tq<float, 1>(epi, N, n, mfma) : shape_tq<double, 1>(epi, N, n, mfma);
    case 2: return fp32 ? shape_tq<float, 2>(epi, N, n, mfma) : shape_tq<double, 2>(epi, N, n, mfma);
    case 4: return fp32 ? shape_tq<float, 4>(epi, N, n, mfma) : shape_tq<double, 4>(epi, N, n, mfma);
  }
  return ApplyShape{-1, 0, 0, 0};
}

hipError_t launch_apply(const OpTab& tab, bool fp32, const ApplyArgs& a, hipStream_t s) {
  // shape checks: the launch shapes above assume these
  if (a.N != tab.q * a.n || a.N < 4 || (a.N & (a.N - 1)) != 0 || a.n > apply_max_elements_x(tab.q))
    return hipErrorInvalidValue;
  switch (tab.q) {
    case 1: return fp32 ? launch_tq<float, 1>(tab, a, s) : launch_tq<double, 1>(tab, a, s);
    case 2: return fp32 ? launch_tq<float, 2>(tab, a, s) : launch_tq<double, 2>(tab, a, s);
    case 4: return fp32 ? launch_tq<float, 4>(tab, a, s) : launch_tq<double, 4>(tab, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gmg
