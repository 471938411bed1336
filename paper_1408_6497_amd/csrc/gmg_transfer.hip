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
#include <map>
#include <mutex>
#include <tuple>

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

// Restriction in one pass over the fine grid (the three axis passes above, fused):
// rc = Rz Ry Rx rf with the same arithmetic -- the x and y results rounded to T as
// the axis passes store them, the z sums taken in FP64 in the same tap order -- so
// the coarse values are the bits of the three-pass restriction.
//   * a block takes full coarse x-rows, blockDim.y coarse rows Y0 .. (one per
//     thread row; a multiple of q) and TZE coarse elements in z; thread (tx, ty)
//     owns coarse element tx in x (q nodes) of coarse row Y0 + ty;
//   * it streams the fine planes of its z window in order: per plane, the x pass
//     of the 2 TY + 2q + 1 fine rows its coarse rows reach goes to LDS, then each
//     thread's y pass gives its q values of that plane;
//   * fine plane 2q E + t' (0 <= t' < 2q) feeds coarse element E at tap 2q + t',
//     the vertex of element E + 1 at tap t', and for t' = 0 element E - 1 at its
//     last tap 4q, which completes that element: three rolling accumulators;
//   * blocks are remapped so that each XCD sweeps a contiguous range of tiles
//     (neighbouring tiles share their halo rows and planes in its L2).
template <typename T, int Q>
__global__ void __launch_bounds__(256) k_restrict3(const T* __restrict__ rf, T* __restrict__ rc,
                                                    const TransferTab tab, const int Nc, const int TZE,
                                                    const int ntiles_y) {
  using V = VecK<T, Q>;
  using V2 = VecK<T, 2 * Q>;
  // fine rows per thread and plane: ceil((2 TY + 2q + 1) / TY) <= 5 for TY >= q
  constexpr int kMaxR = 5;
  const int Nf = 2 * Nc;
  const int nfm = Nf - 1;
  const int ncm = Nc - 1;
  const int TY = blockDim.y;
  const int NFR = 2 * TY + 2 * Q + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* xr = reinterpret_cast<T*>(smem_raw);  // [NFR][Nc]: x-restricted rows of one fine plane
  const int nb = gridDim.x;
  int b = blockIdx.x;
  if ((nb & 7) == 0) b = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  const int Y0 = (b % ntiles_y) * TY;
  const int Z0 = (b / ntiles_y) * TZE;
  const int tx = threadIdx.x;
  const int ty = threadIdx.y;
  const int fy0 = 2 * Y0 - 2 * Q;  // fine row of xr row 0 (wrapped when read)
  const int ay = (Y0 + ty) % Q;    // node class of this thread's coarse row
  const int ey = ty / Q;           // its element within the tile (Y0 is a multiple of q)
  // offsets inside a fine plane of this thread's rows: left vector, right vector, far vertex
  int off_l[kMaxR], off_r[kMaxR], off_f[kMaxR];
#pragma unroll
  for (int k = 0; k < kMaxR; ++k) {
    const int r = ty + k * TY;
    const size_t row = static_cast<size_t>((fy0 + (r < NFR ? r : 0) + Nf) & nfm) * Nf;
    off_l[k] = static_cast<int>(row) + ((2 * Q * tx - 2 * Q + Nf) & nfm);
    off_r[k] = static_cast<int>(row) + 2 * Q * tx;
    off_f[k] = static_cast<int>(row) + ((2 * Q * tx + 2 * Q) & nfm);
  }
  V2 pl[kMaxR], pr[kMaxR];
  T pf[kMaxR];
  const int f0 = 2 * Q * (Z0 - 1);      // first fine plane of the window
  const int total = 2 * Q * (TZE + 1) + 1;
  auto load_plane = [&](int p) {
    const T* plane = rf + static_cast<size_t>((f0 + p + Nf) & nfm) * Nf * Nf;
#pragma unroll
    for (int k = 0; k < kMaxR; ++k) {
      if (ty + k * TY < NFR) {
        pl[k] = *reinterpret_cast<const V2*>(plane + off_l[k]);
        pr[k] = *reinterpret_cast<const V2*>(plane + off_r[k]);
        pf[k] = plane[off_f[k]];
      }
    }
  };
  double P[Q][Q], C[Q][Q], N0[Q];
#pragma unroll
  for (int c = 0; c < Q; ++c) {
    N0[c] = 0.0;
#pragma unroll
    for (int a = 0; a < Q; ++a) P[c][a] = C[c][a] = 0.0;
  }
  load_plane(0);
  for (int p = 0; p < total; ++p) {
    const int tp = p & (2 * Q - 1);
    const int Ef = Z0 - 1 + p / (2 * Q);
    V2 cl[kMaxR], cr[kMaxR];
    T cf[kMaxR];
#pragma unroll
    for (int k = 0; k < kMaxR; ++k) {
      cl[k] = pl[k];
      cr[k] = pr[k];
      cf[k] = pf[k];
    }
    if (p + 1 < total) load_plane(p + 1);  // in flight while this plane is reduced
    // x pass: fine nodes 2qE-2q .. 2qE+2q of coarse element E = tx in each of the rows
#pragma unroll
    for (int k = 0; k < kMaxR; ++k) {
      const int r = ty + k * TY;
      if (r >= NFR) continue;
      T f[4 * Q + 1];
#pragma unroll
      for (int t = 0; t < 2 * Q; ++t) {
        f[t] = cl[k].v[t];
        f[2 * Q + t] = cr[k].v[t];
      }
      f[4 * Q] = cf[k];
      V cv;
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        double sx = 0.0;
#pragma unroll
        for (int t = 0; t <= 4 * Q; ++t) {
          if (a > 0 && t < 2 * Q) continue;
          sx = fma(tab.r[a][t], static_cast<double>(f[t]), sx);
        }
        cv.v[a] = static_cast<T>(sx);
      }
      *reinterpret_cast<V*>(xr + r * Nc + Q * tx) = cv;
    }
    __syncthreads();
    // y pass of this thread's coarse row, then the z taps of this plane
    double sy[Q];
#pragma unroll
    for (int c = 0; c < Q; ++c) sy[c] = 0.0;
#pragma unroll
    for (int t = 0; t <= 4 * Q; ++t) {
      if (ay > 0 && t < 2 * Q) continue;
      const V xv = *reinterpret_cast<const V*>(xr + (2 * Q * ey + t) * Nc + Q * tx);
      const double w = tab.r[ay][t];
#pragma unroll
      for (int c = 0; c < Q; ++c) sy[c] = fma(w, static_cast<double>(xv.v[c]), sy[c]);
    }
#pragma unroll
    for (int c = 0; c < Q; ++c) {
      const double v = static_cast<double>(static_cast<T>(sy[c]));
      if (tp == 0) {
#pragma unroll
        for (int a = 0; a < Q; ++a) P[c][a] = fma(tab.r[a][4 * Q], v, P[c][a]);
      }
#pragma unroll
      for (int a = 0; a < Q; ++a) C[c][a] = fma(tab.r[a][2 * Q + tp], v, C[c][a]);
      N0[c] = fma(tab.r[0][tp], v, N0[c]);
    }
    if (tp == 0 && Ef - 1 >= Z0) {
      // element Ef - 1 is complete: its q coarse planes
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        V out;
#pragma unroll
        for (int c = 0; c < Q; ++c) out.v[c] = static_cast<T>(P[c][a]);
        const int kz = (Q * (Ef - 1) + a) & ncm;
        *reinterpret_cast<V*>(rc + (static_cast<size_t>(kz) * Nc + Y0 + ty) * Nc + Q * tx) = out;
      }
    }
    __syncthreads();  // xr is refilled by the next plane
    if (tp == 2 * Q - 1) {
      // element Ef becomes the one completed next, element Ef + 1 the one being filled
#pragma unroll
      for (int c = 0; c < Q; ++c) {
#pragma unroll
        for (int a = 0; a < Q; ++a) P[c][a] = C[c][a];
        C[c][0] = N0[c];
#pragma unroll
        for (int a = 1; a < Q; ++a) C[c][a] = 0.0;
        N0[c] = 0.0;
      }
    }
  }
}

// Prolongation in one pass: uf += Pz Py Px ec with the arithmetic of the three axis
// passes (x and y results rounded to T, the z sum in FP64 added to uf in FP64 and
// rounded), so uf gets the bits of the three-pass prolongation.
//   * a block takes full fine x-rows, 2 blockDim.y fine rows (whole coarse elements
//     in y: blockDim.y is a multiple of q) and TZE coarse elements in z; thread
//     (tx, ty) owns the 2q fine x nodes of coarse element tx in fine rows 2 ty and
//     2 ty + 1 of the tile;
//   * per coarse element E in z: the x pass of its q+1 coarse planes over the
//     tile's coarse rows goes to LDS; each thread then forms its rows' y values on
//     those q+1 planes and the 2q fine planes of E from them, added into uf.
template <typename T, int Q>
__global__ void __launch_bounds__(256) k_prolong3(const T* __restrict__ ec, T* __restrict__ uf,
                                                   const TransferTab tab, const int Nc, const int TZE,
                                                   const int ntiles_y) {
  using V = VecK<T, Q>;
  using V2 = VecK<T, 2 * Q>;
  constexpr int kRows = 2;  // fine rows per thread
  const int Nf = 2 * Nc;
  const int ncm = Nc - 1;
  const int TY = blockDim.y;
  const int TYF = kRows * TY;        // fine rows of the tile
  const int NCR = TYF / 2 + 1;       // coarse rows they reach: whole elements plus the closing vertex
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* xp = reinterpret_cast<T*>(smem_raw);  // [q+1 planes][NCR][Nf]: x-prolonged coarse rows
  const int nb = gridDim.x;
  int b = blockIdx.x;
  if ((nb & 7) == 0) b = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
  const int Y0 = (b % ntiles_y) * TYF;  // first fine row (a multiple of 2q)
  const int Z0 = (b / ntiles_y) * TZE;
  const int tx = threadIdx.x;
  const int ty = threadIdx.y;
  const int cy0 = Y0 / 2;               // first coarse row
  for (int E = Z0; E < Z0 + TZE; ++E) {
    // x pass: coarse nodes qE' .. qE'+q of element E' = tx on plane qE + a, coarse row cy0 + r
    for (int it = ty; it < (Q + 1) * NCR; it += TY) {
      const int a = it / NCR;
      const int r = it - a * NCR;
      const T* row = ec + (static_cast<size_t>((Q * E + a) & ncm) * Nc + ((cy0 + r) & ncm)) * Nc;
      T c[Q + 1];
      const V cv = *reinterpret_cast<const V*>(row + Q * tx);
#pragma unroll
      for (int k = 0; k < Q; ++k) c[k] = cv.v[k];
      c[Q] = row[(Q * tx + Q) & ncm];
      V2 fv;
#pragma unroll
      for (int bb = 0; bb < 2 * Q; ++bb) {
        double sx = 0.0;
#pragma unroll
        for (int k = 0; k <= Q; ++k) sx = fma(tab.p[bb][k], static_cast<double>(c[k]), sx);
        fv.v[bb] = static_cast<T>(sx);
      }
      *reinterpret_cast<V2*>(xp + (a * NCR + r) * Nf + 2 * Q * tx) = fv;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRows; ++i) {
      const int fr = kRows * ty + i;        // fine row within the tile
      const int ey = fr / (2 * Q);          // its coarse element in y, within the tile
      const int by = fr - 2 * Q * ey;       // and its child index there
      // y values of this row on the q+1 coarse planes, rounded as the y pass stores them
      T xy[Q + 1][2 * Q];
#pragma unroll
      for (int a = 0; a <= Q; ++a) {
        double sy[2 * Q];
#pragma unroll
        for (int t = 0; t < 2 * Q; ++t) sy[t] = 0.0;
#pragma unroll
        for (int k = 0; k <= Q; ++k) {
          const V2 v = *reinterpret_cast<const V2*>(xp + (a * NCR + Q * ey + k) * Nf + 2 * Q * tx);
          const double w = tab.p[by][k];
#pragma unroll
          for (int t = 0; t < 2 * Q; ++t) sy[t] = fma(w, static_cast<double>(v.v[t]), sy[t]);
        }
#pragma unroll
        for (int t = 0; t < 2 * Q; ++t) xy[a][t] = static_cast<T>(sy[t]);
      }
#pragma unroll
      for (int bz = 0; bz < 2 * Q; ++bz) {
        T* o = uf + (static_cast<size_t>(2 * Q * E + bz) * Nf + (Y0 + fr)) * Nf + 2 * Q * tx;
        V2 u = *reinterpret_cast<const V2*>(o);
#pragma unroll
        for (int t = 0; t < 2 * Q; ++t) {
          double sz = 0.0;
#pragma unroll
          for (int a = 0; a <= Q; ++a) sz = fma(tab.p[bz][a], static_cast<double>(xy[a][t]), sz);
          u.v[t] = static_cast<T>(static_cast<double>(u.v[t]) + sz);
        }
        *reinterpret_cast<V2*>(o) = u;
      }
    }
    __syncthreads();  // xp is refilled for the next element
  }
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

// Launch shape of the fused restriction onto Nc coarse nodes a side: coarse rows per
// block (one per thread row, about 256 threads a block), and the z chunk TZE that
// minimises rounds x fine planes per block, 2q (TZE + 1) + 1, given the blocks the
// device holds at once (occupancy, cached; primed at setup so that no query runs
// during graph capture).
struct R3Shape {
  int TY, TZE, ntiles_y, nblocks;
  size_t lds;
};

template <typename T, int Q>
R3Shape r3_shape(int Nc) {
  R3Shape sh{};
  const int nxc = Nc / Q;
  int TY = 256 / nxc;
  if (TY < Q) TY = Q;
  if (TY > Nc) TY = Nc;
  sh.TY = TY;
  sh.ntiles_y = Nc / TY;
  sh.lds = static_cast<size_t>(2 * TY + 2 * Q + 1) * Nc * sizeof(T);
  static std::mutex mu;
  static std::map<std::tuple<int, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  int resident = 0;
  {
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_tuple(dev, Nc);
    const auto it = cache.find(key);
    if (it != cache.end()) {
      resident = it->second;
    } else {
      int per_cu = 0, cus = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_restrict3<T, Q>),
                                                       nxc * TY, sh.lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
      (void)hipGetLastError();
      resident = cache[key] = per_cu * cus;
    }
  }
  const int ne = Nc / Q;
  int best = 1;
  int64_t best_cost = -1;
  for (int tz = 1; tz <= ne; tz <<= 1) {
    const int64_t blocks = static_cast<int64_t>(sh.ntiles_y) * (ne / tz);
    const int64_t cost = (blocks + resident - 1) / resident * (2 * Q * (tz + 1) + 1);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = tz;
    }
  }
  sh.TZE = best;
  sh.nblocks = sh.ntiles_y * (ne / best);
  return sh;
}

template <typename T, int Q>
hipError_t restrict3_fused(const TransferTab& tab, const T* rf, T* rc, int Nc, hipStream_t s) {
  const R3Shape sh = r3_shape<T, Q>(Nc);
  if (Nc % sh.TY != 0 || sh.TY % Q != 0 || (Nc / Q) * sh.TY > 256) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_restrict3<T, Q>), dim3(sh.nblocks), dim3(Nc / Q, sh.TY), sh.lds, s, rf, rc, tab, Nc, sh.TZE,
                     sh.ntiles_y);
  return hipGetLastError();
}

template <typename T>
hipError_t restrict_fused_q(int q, const TransferTab& tab, const T* rf, T* rc, int Nc, hipStream_t s) {
  switch (q) {
    case 1: return restrict3_fused<T, 1>(tab, rf, rc, Nc, s);
    case 2: return restrict3_fused<T, 2>(tab, rf, rc, Nc, s);
    case 4: return restrict3_fused<T, 4>(tab, rf, rc, Nc, s);
  }
  return hipErrorInvalidValue;
}

// Launch shape of the fused prolongation from Nc coarse nodes a side: about 256
// threads, 2 fine rows per thread row, and the z chunk that minimises rounds x
// elements per block (occupancy cached and primed at setup like the restriction's).
template <typename T, int Q>
R3Shape p3_shape(int Nc) {
  R3Shape sh{};
  const int nxc = Nc / Q;
  int TY = 256 / nxc;
  if (TY < Q) TY = Q;
  if (TY > Nc) TY = Nc;  // 2 TY fine rows <= 2 Nc
  sh.TY = TY;
  sh.ntiles_y = (2 * Nc) / (2 * TY);
  sh.lds = static_cast<size_t>(Q + 1) * (TY + 1) * (2 * Nc) * sizeof(T);
  static std::mutex mu;
  static std::map<std::tuple<int, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  int resident = 0;
  {
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_tuple(dev, Nc);
    const auto it = cache.find(key);
    if (it != cache.end()) {
      resident = it->second;
    } else {
      int per_cu = 0, cus = 0;
      const void* fn = reinterpret_cast<const void*>(&k_prolong3<T, Q>);
      if (sh.lds > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                    static_cast<int>(sh.lds));
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, nxc * TY, sh.lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
      (void)hipGetLastError();
      resident = cache[key] = per_cu * cus;
    }
  }
  const int ne = Nc / Q;
  int best = 1;
  int64_t best_cost = -1;
  for (int tz = 1; tz <= ne; tz <<= 1) {
    const int64_t blocks = static_cast<int64_t>(sh.ntiles_y) * (ne / tz);
    const int64_t cost = (blocks + resident - 1) / resident * tz;
    if (best_cost < 0 || cost <= best_cost) {  // ties: the longer chunk
      best_cost = cost;
      best = tz;
    }
  }
  sh.TZE = best;
  sh.nblocks = sh.ntiles_y * (ne / best);
  return sh;
}

template <typename T, int Q>
hipError_t prolong3_fused(const TransferTab& tab, const T* ec, T* uf, int Nc, hipStream_t s) {
  const R3Shape sh = p3_shape<T, Q>(Nc);
  if ((2 * sh.TY) % (2 * Q) != 0 || (2 * Nc) % (2 * sh.TY) != 0 || (Nc / Q) * sh.TY > 256)
    return hipErrorInvalidConfiguration;
  if (sh.lds > 65536) {  // q = 4 in FP64: up to 102 KB of the 160 KB a CU has
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_prolong3<T, Q>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(sh.lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_prolong3<T, Q>), dim3(sh.nblocks), dim3(Nc / Q, sh.TY), sh.lds, s, ec, uf, tab, Nc, sh.TZE,
                     sh.ntiles_y);
  return hipGetLastError();
}

template <typename T>
hipError_t prolong_fused_q(int q, const TransferTab& tab, const T* ec, T* uf, int Nc, hipStream_t s) {
  switch (q) {
    case 1: return prolong3_fused<T, 1>(tab, ec, uf, Nc, s);
    case 2: return prolong3_fused<T, 2>(tab, ec, uf, Nc, s);
    case 4: return prolong3_fused<T, 4>(tab, ec, uf, Nc, s);
  }
  return hipErrorInvalidValue;
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

// one thread per coarse element of a row, q coarse rows at least: 256 threads hold
// Nc <= 256; q = 4 keeps the axis passes (measured slower fused on every level but
// the finest, 18.6 against 13.9 us from 16^3 coarse nodes)
bool prolong_fusable(int q, int Nc) { return q <= 2 && Nc >= 2 * q && Nc <= 256; }

hipError_t launch_prolong(const TransferTab& tab, bool fp32, const void* ec, void* t1, void* t2, void* uf, int Nc,
                          hipStream_t s, bool fused) {
  if (Nc < tab.q || (Nc & (Nc - 1)) != 0 || Nc > 1024) return hipErrorInvalidValue;
  if (fused && prolong_fusable(tab.q, Nc)) {
    if (fp32) return prolong_fused_q<float>(tab.q, tab, static_cast<const float*>(ec), static_cast<float*>(uf), Nc, s);
    return prolong_fused_q<double>(tab.q, tab, static_cast<const double*>(ec), static_cast<double*>(uf), Nc, s);
  }
  if (fp32)
    return prolong_q<float>(tab.q, tab, static_cast<const float*>(ec), static_cast<float*>(t1),
                            static_cast<float*>(t2), static_cast<float*>(uf), Nc, s);
  return prolong_q<double>(tab.q, tab, static_cast<const double*>(ec), static_cast<double*>(t1),
                           static_cast<double*>(t2), static_cast<double*>(uf), Nc, s);
}

// One thread per coarse element of a row, q coarse rows at least: 256 threads hold
// Nc <= 256.  Below 64 coarse nodes a side the chain of 2q (TZE + 1) + 1 fine planes
// a block streams is longer than the three short axis launches (measured: 14-15 us
// against 11.5 us onto 16^3 and 32^3 nodes, q = 2), so those keep the axis passes.
// q = 4 keeps the axis passes: its 4q+1-tap windows make the halo rows and planes
// cost more than the passes they replace (measured onto 128^3 nodes: 85 against
// 54 us, the Q4 solve 10.65 against 10.44 ms).
bool restrict_fusable(int q, int Nc) { return q <= 2 && Nc >= 64 && Nc >= 2 * q && Nc <= 256; }

void prime_transfer_shapes(int q, int Nc) {
  if (prolong_fusable(q, Nc)) {
    switch (q) {
      case 1: p3_shape<float, 1>(Nc); p3_shape<double, 1>(Nc); break;
      case 2: p3_shape<float, 2>(Nc); p3_shape<double, 2>(Nc); break;
      case 4: p3_shape<float, 4>(Nc); p3_shape<double, 4>(Nc); break;
    }
  }
  if (!restrict_fusable(q, Nc)) return;
  switch (q) {
    case 1: r3_shape<float, 1>(Nc); r3_shape<double, 1>(Nc); break;
    case 2: r3_shape<float, 2>(Nc); r3_shape<double, 2>(Nc); break;
    case 4: r3_shape<float, 4>(Nc); r3_shape<double, 4>(Nc); break;
  }
}

hipError_t launch_restrict(const TransferTab& tab, bool fp32, const void* rf, void* t1, void* t2, void* rc, int Nc,
                           hipStream_t s, bool fused) {
  if (Nc < tab.q || (Nc & (Nc - 1)) != 0 || Nc > 1024) return hipErrorInvalidValue;
  if (fused && restrict_fusable(tab.q, Nc)) {
    if (fp32)
      return restrict_fused_q<float>(tab.q, tab, static_cast<const float*>(rf), static_cast<float*>(rc), Nc, s);
    return restrict_fused_q<double>(tab.q, tab, static_cast<const double*>(rf), static_cast<double*>(rc), Nc, s);
  }
  if (fp32)
    return restrict_q<float>(tab.q, tab, static_cast<const float*>(rf), static_cast<float*>(t1),
                             static_cast<float*>(t2), static_cast<float*>(rc), Nc, s);
  return restrict_q<double>(tab.q, tab, static_cast<const double*>(rf), static_cast<double*>(t1),
                            static_cast<double*>(t2), static_cast<double*>(rc), Nc, s);
}

}  // namespace gmg
