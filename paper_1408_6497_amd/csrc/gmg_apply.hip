// Matrix-free, sum-factorized Q_q stiffness apply on uniform periodic meshes
// (Section 2.3.2: tensorized LGL nodal basis, element MatVec in O(q^4) instead
// of O(q^6); here the tensor structure is used globally, so each node is
// touched once per 1D pass).
//
// Operator:  A = Kx (x) My (x) Mz + Mx (x) Ky (x) Mz + Mx (x) My (x) Kz
// split per z plane:  g = (Kx My + Mx Ky) x,  h = Mx My x,  A x = Mz g + Kz h.
//
// Work decomposition (gfx950, 64-wide wavefronts):
//   * a workgroup owns a tile of TY = 4*G full x-rows and a chunk of TZ element
//     layers in z; thread (tx, ty) owns one element column in x (q nodes,
//     loaded/stored as one q-wide vector, so a wavefront streams 64*q
//     consecutive values per row) and RY = 4 rows;
//   * each input plane is staged once in LDS with a q-row halo in y (rows
//     wrap periodically), the y pass writes (My x, Ky x) for the TY rows back
//     to LDS, the x pass reads the neighbouring element columns from LDS
//     (periodic wrap) and produces (g, h) in registers;
//   * the z pass is done element layer by element layer with q+1 register
//     accumulators per point (element form), so only one plane of halo
//     (the vertex plane below the chunk) is recomputed per element layer;
//   * the next plane's global loads are issued before the LDS passes of the
//     current plane (one-plane register prefetch);
//   * node classes (i mod q) are compile-time in y and z and per thread in x,
//     so banded taps that are structurally zero are never issued;
//   * blocks are remapped so that each XCD (blockIdx mod 8) sweeps a
//     contiguous range of tiles and shares halos in its own L2.
// Epilogues fuse the residual (b - A x) and the Chebyshev-Jacobi step
// x + c1 (x - x_prev) + c2 D^-1 (b - A x) into the same pass.
#include "gmg_kernels.h"

namespace gmg {
namespace {

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
  T dinv[Q * Q * Q];
};

// Is offset o (in -Q..Q) a structural nonzero of the assembled 1D row of class c?
__host__ __device__ constexpr bool tap(int Q, int c, int o) {
  return c == 0 ? true : (o >= -c && o <= Q - c);
}

template <typename T, int Q, int G, int EPI>
__global__ void __launch_bounds__(512) k_apply(const T* __restrict__ x, const KTab<T, Q> tb, const int N,
                                                 const int TZ, const int ntiles_y, T* out, const T* bvec,
                                                 const T* xp, const T c1, const T c2) {
  constexpr int RY = 4;
  constexpr int TY = G * RY;
  constexpr int NR = TY + 2 * Q;
  constexpr int NL = (NR + G - 1) / G;
  using V = VecQ<T, Q>;

  const int tx = threadIdx.x;
  const int ty = threadIdx.y;
  const int NX = N / Q;
  const int Nm = N - 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* xs = reinterpret_cast<T*>(smem_raw);  // NR x N
  T* ps = xs + NR * N;                     // TY x N
  T* ss = ps + TY * N;                     // TY x N

  const int nblocks = gridDim.x;
  int tile = blockIdx.x;
  if ((nblocks & 7) == 0) tile = (blockIdx.x & 7) * (nblocks >> 3) + (blockIdx.x >> 3);
  const int Y0 = (tile % ntiles_y) * TY;
  const int E0 = (tile / ntiles_y) * TZ;
  const size_t NN = static_cast<size_t>(N) * N;

  V pre[NL];
  auto load_plane = [&](int p) {
    const T* base = x + static_cast<size_t>(p & Nm) * NN;
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int r = ty + i * G;
      if (r < NR) {
        const int yy = (Y0 - Q + r) & Nm;
        pre[i] = *reinterpret_cast<const V*>(base + static_cast<size_t>(yy) * N + Q * tx);
      }
    }
  };
  auto store_plane = [&]() {
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int r = ty + i * G;
      if (r < NR) *reinterpret_cast<V*>(xs + r * N + Q * tx) = pre[i];
    }
  };

  T g[RY][Q], h[RY][Q];
  const int txl = (tx - 1) & (NX - 1);
  const int txr = (tx + 1) & (NX - 1);

  auto compute_gh = [&](int p, bool prefetch) {
    store_plane();
    if (prefetch) load_plane(p + 1);
    __syncthreads();
    // ---- y pass: P = My x, S = Ky x on this thread's RY rows and q columns
    {
      V xv[RY + 2 * Q];
#pragma unroll
      for (int r = 0; r < RY + 2 * Q; ++r) xv[r] = *reinterpret_cast<const V*>(xs + (ty * RY + r) * N + Q * tx);
#pragma unroll
      for (int i = 0; i < RY; ++i) {
        const int ci = i % Q;
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
    }
    __syncthreads();
    // ---- x pass: g = Kx P + Mx S, h = Mx P
#pragma unroll
    for (int i = 0; i < RY; ++i) {
      const int row = (ty * RY + i) * N;
      T pw[3 * Q], sw[3 * Q];
      {
        const V a = *reinterpret_cast<const V*>(ps + row + Q * txl);
        const V b = *reinterpret_cast<const V*>(ps + row + Q * tx);
        const V c = *reinterpret_cast<const V*>(ps + row + Q * txr);
        const V d = *reinterpret_cast<const V*>(ss + row + Q * txl);
        const V e = *reinterpret_cast<const V*>(ss + row + Q * tx);
        const V f = *reinterpret_cast<const V*>(ss + row + Q * txr);
#pragma unroll
        for (int c2i = 0; c2i < Q; ++c2i) {
          pw[c2i] = a.v[c2i];
          pw[Q + c2i] = b.v[c2i];
          pw[2 * Q + c2i] = c.v[c2i];
          sw[c2i] = d.v[c2i];
          sw[Q + c2i] = e.v[c2i];
          sw[2 * Q + c2i] = f.v[c2i];
        }
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
  };

  T acc[RY][Q][Q + 1];
  const int zlast = (E0 + TZ) * Q;  // last plane of the chunk (vertex plane above it)

  load_plane((E0 - 1) * Q);
  compute_gh((E0 - 1) * Q, true);
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
      compute_gh(p, p < zlast);
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
          const size_t idx = zoff + static_cast<size_t>(Y0 + ty * RY + i) * N + Q * tx;
          V res;
          if constexpr (EPI == static_cast<int>(Epi::Apply)) {
#pragma unroll
            for (int c = 0; c < Q; ++c) res.v[c] = acc[i][c][a];
          } else if constexpr (EPI == static_cast<int>(Epi::Residual)) {
            const V bv = *reinterpret_cast<const V*>(bvec + idx);
#pragma unroll
            for (int c = 0; c < Q; ++c) res.v[c] = bv.v[c] - acc[i][c][a];
          } else {
            const V bv = *reinterpret_cast<const V*>(bvec + idx);
            const V xv = *reinterpret_cast<const V*>(x + idx);
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
            const int ci = i % Q;
#pragma unroll
            for (int c = 0; c < Q; ++c) {
              const T dinv = tb.dinv[c + Q * (ci + Q * a)];
              const T rr = bv.v[c] - acc[i][c][a];
              res.v[c] = xv.v[c] + c1 * (xv.v[c] - pv.v[c]) + c2 * dinv * rr;
            }
          }
          *reinterpret_cast<V*>(out + idx) = res;
        }
      }
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

inline size_t apply_lds(int G, int Q, int N, size_t elem) {
  return static_cast<size_t>(12 * G + 2 * Q) * N * elem;
}

inline size_t max_lds_per_block() {
  static size_t cached = 0;
  if (cached == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
      cached = static_cast<size_t>(v);
    else
      cached = 65536;
  }
  return cached;
}

template <typename T, int Q>
KTab<T, Q> make_ktab(const OpTab& t) {
  KTab<T, Q> k{};
  for (int c = 0; c < Q; ++c)
    for (int o = 0; o < 2 * Q + 1; ++o) {
      k.kr[c][o] = static_cast<T>(t.krow[c][o]);
      k.mr[c][o] = static_cast<T>(t.mrow[c][o]);
    }
  for (int a = 0; a <= Q; ++a)
    for (int b = 0; b <= Q; ++b) {
      k.zk[a][b] = static_cast<T>(t.zk[a][b]);
      k.zm[a][b] = static_cast<T>(t.zm[a][b]);
    }
  for (int i = 0; i < Q * Q * Q; ++i) k.dinv[i] = static_cast<T>(t.dinv[i]);
  return k;
}

template <typename T, int Q, int G, int EPI>
hipError_t launch_tq(const OpTab& tab, const ApplyArgs& a, hipStream_t s) {
  constexpr int TY = 4 * G;
  const int N = a.N;
  const int n = a.n;
  const int ntiles_y = N / TY;
  // element layers per block: enough blocks to fill 256 CUs several times while
  // keeping the recomputed layer below the chunk small
  int TZ = n;
  while (TZ > 2 && static_cast<int64_t>(ntiles_y) * (n / TZ) < 2048) TZ >>= 1;
  const int nchunks = n / TZ;
  const dim3 block(N / Q, G);
  const dim3 grid(ntiles_y * nchunks);
  const size_t lds = apply_lds(G, Q, N, sizeof(T));
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_apply<T, Q, G, EPI>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  const KTab<T, Q> kt = make_ktab<T, Q>(tab);
  hipLaunchKernelGGL((k_apply<T, Q, G, EPI>), grid, block, lds, s, static_cast<const T*>(a.x), kt, N, TZ,
                     ntiles_y, static_cast<T*>(a.out), static_cast<const T*>(a.b), static_cast<const T*>(a.xp),
                     static_cast<T>(a.c1), static_cast<T>(a.c2));
  return hipGetLastError();
}

template <typename T, int Q, int G>
hipError_t launch_tqg(const OpTab& tab, const ApplyArgs& a, hipStream_t s) {
  switch (a.epi) {
    case Epi::Apply: return launch_tq<T, Q, G, 0>(tab, a, s);
    case Epi::Residual: return launch_tq<T, Q, G, 1>(tab, a, s);
    case Epi::Cheb: return launch_tq<T, Q, G, 2>(tab, a, s);
  }
  return hipErrorInvalidValue;
}

// Row groups per block: as many as fit 512 threads and the LDS budget, with
// TY = 4 G rows dividing N.  Returns 0 when even G = 1 does not fit.
inline int pick_g(int N, int Q, size_t elem) {
  const int nx = N / Q;
  const size_t lim = max_lds_per_block();
  for (int G = 4; G >= 1; G >>= 1)
    if (G * nx <= 512 && 4 * G <= N && apply_lds(G, Q, N, elem) <= lim) return G;
  return 0;
}

template <typename T, int Q>
hipError_t launch_tqx(const OpTab& tab, const ApplyArgs& a, hipStream_t s) {
  switch (pick_g(a.N, Q, sizeof(T))) {
    case 4: return launch_tqg<T, Q, 4>(tab, a, s);
    case 2: return launch_tqg<T, Q, 2>(tab, a, s);
    case 1: return launch_tqg<T, Q, 1>(tab, a, s);
    default: return hipErrorInvalidConfiguration;
  }
}

}  // namespace

hipError_t launch_apply(const OpTab& tab, bool fp32, const ApplyArgs& a, hipStream_t s) {
  // shape checks: the grid above assumes these
  if (a.N != tab.q * a.n || a.N < 4 || (a.N & (a.N - 1)) != 0 || a.N / tab.q > 512) return hipErrorInvalidValue;
  switch (tab.q) {
    case 1: return fp32 ? launch_tqx<float, 1>(tab, a, s) : launch_tqx<double, 1>(tab, a, s);
    case 2: return fp32 ? launch_tqx<float, 2>(tab, a, s) : launch_tqx<double, 2>(tab, a, s);
    case 4: return fp32 ? launch_tqx<float, 4>(tab, a, s) : launch_tqx<double, 4>(tab, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gmg
