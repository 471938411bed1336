// Host-side interface of the gfx950 kernels of the multigrid hot path.
//
// Every launcher enqueues on the given stream and returns the launch status.
// Level vectors are N^3 DoF vectors, x fastest (index i + N (j + N k)),
// N = q * n with n (elements per direction) a power of two.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace gmg {

constexpr int kMaxQ = 4;
constexpr int kMaxTaps = 4 * kMaxQ + 1;

// Coefficients of the sum-factorized operator on one level (FP64 master copy;
// the launchers convert to the kernel precision).
//   A = Kx (x) My (x) Mz + Mx (x) Ky (x) Mz + Mx (x) My (x) Kz,
// with the x and y passes done by rows of the assembled periodic 1D matrices
// (krow, mrow: node class c = i mod q, offsets -q..q) and the z pass done
// element by element (zk, zm: (q+1) x (q+1) element matrices).
// The same kernels apply the mass M (x) M (x) M with krow = 0, zk = zkrow = mass
// and zm = zmrow = 0.
struct OpTab {
  int q;
  double krow[kMaxQ][2 * kMaxQ + 1];
  double mrow[kMaxQ][2 * kMaxQ + 1];
  double zk[kMaxQ + 1][kMaxQ + 1];
  double zm[kMaxQ + 1][kMaxQ + 1];
  // the same two z operators as assembled periodic rows (used by the point kernel)
  double zkrow[kMaxQ][2 * kMaxQ + 1];
  double zmrow[kMaxQ][2 * kMaxQ + 1];
  double dinv[kMaxQ * kMaxQ * kMaxQ];  // 1 / A_ii by node class (cx + q (cy + q cz))
};

// One-axis transfer weights (P = P1 (x) P1 (x) P1 on uniform meshes).
//   p[b][a]: fine node 2qE + b (b < 2q) from coarse node qE + a (a <= q) of
//            coarse element E: phi_a at the child node;
//   r[a][t]: coarse node qE + a (a < q) from fine node 2qE - 2q + t (t <= 4q);
//            the row of P^T.
struct TransferTab {
  int q;
  double p[2 * kMaxQ][kMaxQ + 1];
  double r[kMaxQ][4 * kMaxQ + 1];
};

enum class Epi : int { Apply = 0, Residual = 1, Cheb = 2, ChebZero = 3, ApplyDot = 4, ResidualSums = 5, ResidualNorms = 6 };

// out = A x                          (Epi::Apply)
// out = A x, sc[d0] = x . A x and sc[d1] = sum(A x)   (Epi::ApplyDot: FP64, uniform levels
//                                      of N >= 64 nodes; per-block partials go to part, which
//                                      must hold twice the block count and their folding)
// out = b - A x, sc[d0] = out . out and sc[d1] = sum(out)   (Epi::ResidualSums: the same
//                                      conditions as Epi::ApplyDot)
// out = b - A x                      (Epi::Residual)
// sc[d0] = |b - A x|^2 and sc[d1] = |b|^2, nothing stored (Epi::ResidualNorms: FP32 or FP64,
//                                      uniform levels of N >= 64 nodes; partials as ApplyDot)
// out = x + c1 (x - xp) + c2 D^-1 (b - A x)   (Epi::Cheb; xp unused when c1 == 0,
//                                      read as zero when null; out may alias xp, never x)
// the first two Chebyshev steps from x_0 = 0 in one pass (Epi::ChebZero, uniform
// levels): x_1 = s0 D^-1 b is formed from b as it is loaded (x must be b), then
// out = x_1 + c1 x_1 + c2 D^-1 (b - A x_1) and x1 = x_1 is stored as well
struct ApplyArgs {
  int N;  // lattice nodes per direction
  int n;  // elements per direction
  const void* x;
  void* out;
  const void* b;
  const void* xp;
  double c1, c2;
  Epi epi;
  void* x1;   // Epi::ChebZero: where x_1 goes
  double s0;  // Epi::ChebZero: x_1 = s0 D^-1 b
  // Epi::ApplyDot: partials buffer (part_cap doubles) and the destination scalar slots
  double* part;
  int64_t part_cap;
  double* sc;
  int d0, d1;
  bool mfma = false;  // FP32 q = 4 column kernel: x and z passes on the matrix cores
};

// Exact FFT solve of the uniform periodic Q1 system on N^3 nodes (FP64): plans and the
// spectrum buffer are made by fft_q1_prepare and kept until the object is destroyed.
struct FftQ1 {
  int N = 0;
  void* fwd = nullptr;  // hipfftHandle (an opaque pointer)
  void* inv = nullptr;
  bool fwd_ok = false, inv_ok = false;
  void* spec = nullptr;
  ~FftQ1();
};
hipError_t fft_q1_prepare(FftQ1* f, int N);
hipError_t fft_q1_solve(FftQ1* f, const double* b, double* u, hipStream_t s);
// The same for uniform periodic Q2 on n^3 elements: 8 node classes, batched FFTs over the
// elements and a 2x2-per-axis eigenbasis of the block symbol (tables on the device).
struct FftQ2 {
  int n = 0;
  void* fwd = nullptr;
  void* inv = nullptr;
  bool fwd_ok = false, inv_ok = false;
  void* spec = nullptr;  // 8 class spectra
  void* cls = nullptr;   // 8 class arrays of n^3 values
  void* axis = nullptr;  // per-wavenumber eigenbasis of one axis
  ~FftQ2();
};
hipError_t fft_q2_prepare(FftQ2* f, int n);
hipError_t fft_q2_solve(FftQ2* f, const double* b, double* u, hipStream_t s);
// Q4: 64 node classes, 4x4 pencils per axis (same members as FftQ2)
struct FftQ4 {
  int n = 0;
  void* fwd = nullptr;
  void* inv = nullptr;
  bool fwd_ok = false, inv_ok = false;
  void* spec = nullptr;
  void* cls = nullptr;
  void* axis = nullptr;
  ~FftQ4();
};
hipError_t fft_q4_prepare(FftQ4* f, int n);
hipError_t fft_q4_solve(FftQ4* f, const double* b, double* u, hipStream_t s);

// Orders without a specialised kernel (q = 3 and 5 .. 16; gmg_generic.hip): the operator as
// three banded 1D passes through four level-size temporaries, transfers as one-axis passes,
// and the node-class arithmetic with its class tables in device memory.
constexpr int kGenMaxQ = 16;
// rows: 6 blocks of q (2q+1) values (z K, z M, y K, y M, x K, x M; row c = node class,
// tap o + q for offset o); dinv: 1 / A_ii by node class (q^3)
struct GenOp {
  int q = 0;
  const double* rows64 = nullptr;
  const float* rows32 = nullptr;
  const double* dinv64 = nullptr;
  const float* dinv32 = nullptr;
};
// p: 2q x (q+1) weights of P1, r: q x (4q+1) weights of P1^T (device, FP64), laid out as
// the one-axis tables of TransferTab
struct GenXfer {
  int q = 0;
  const double* p = nullptr;
  const double* r = nullptr;
};
// Epi::Apply, Residual and Cheb (the fused variants are for q = 1, 2, 4); tmp: four
// temporaries of N^3 values of the kernel precision
hipError_t launch_gen_apply(const GenOp& op, bool fp32, const ApplyArgs& a, void* const tmp[4], hipStream_t s);
hipError_t launch_gen_prolong(const GenXfer& t, bool fp32, const void* ec, void* t1, void* t2, void* uf, int Nc,
                              hipStream_t s);
hipError_t launch_gen_restrict(const GenXfer& t, bool fp32, const void* rf, void* t1, void* t2, void* rc, int Nc,
                               hipStream_t s);
// out = c tab[class] in (in null: 1; tab null: 1); v += c tab[class] (FP64); dst = sum tab[class] x
hipError_t launch_gclass_scale(bool fp32, int q, int N, const double* tab_dev, double c, const void* in, void* out,
                               hipStream_t s);
hipError_t launch_gclass_axpy(int q, int N, const double* tab_dev, double c, double* v, hipStream_t s);
hipError_t launch_gclass_dot(bool fp32, int q, int N, const double* tab_dev, const void* x, double* part,
                             int64_t part_cap, double* dst, hipStream_t s);

// Spectral FFT Poisson solve on the uniform N^3 grid (16 <= N <= 1024, a power of two):
// u = F^-1 [F(f) / (4 pi^2 |m|^2)] with the m = 0 coefficient set to 0.  The complex
// work buffer (N^3 values) and the table of the N roots of unity are made by
// spectral_prepare and kept until the object is destroyed; f and u may alias.
struct FftSpectral {
  int N = 0;
  void* buf = nullptr;
  void* tw = nullptr;
  ~FftSpectral();
};
bool spectral_size_ok(int N);
hipError_t spectral_prepare(FftSpectral* s, int N);
hipError_t spectral_solve(const FftSpectral& s, const double* f, double* u, hipStream_t st);

hipError_t launch_apply(const OpTab& tab, bool fp32, const ApplyArgs& a, hipStream_t s);
// The launch shape launch_apply takes on a uniform level: kernel 0 = the point kernel
// (N <= 32), 1 = the streaming column kernel, 2 = the column kernel that loads all the
// planes of its one-layer z chunk at once, 3 the streaming column kernel with its x and z
// passes on the matrix cores (mfma: FP32 q = 4 only); G (4G rows per tile), TZ (element
// layers per block, 0 for the point kernel) and the block count.  kernel = -1 for an
// unsupported combination.
struct ApplyShape {
  int kernel, G, TZ, nblocks;
};
ApplyShape apply_shape(int q, bool fp32, Epi epi, int N, int n, bool mfma = false);
// Query (once per device) the occupancy that the launch shape of every apply
// kernel instance for a level of N nodes a side depends on; call before any
// launch sequence is captured into a graph.
void prime_apply_shapes(int q, int N);

// Device arrays of one octree level (owned by the library context).  The
// stiffness is C^T blockdiag(h_e kref) C and the mass C^T blockdiag(h_e^3 mref) C,
// with C the element-node constraint map (E m rows, CSR) and h_e = 2^-lev[e].
struct OctLevelDev {
  int64_t E = 0;  // leaves
  int64_t n = 0;  // DoFs
  int m = 0;      // nodes per element, (q+1)^3 (8 or 27)
  const uint8_t* lev = nullptr;
  const int* cptr = nullptr;
  const int* ccol = nullptr;
  const double* cval64 = nullptr;
  const float* cval32 = nullptr;
  const int* tptr = nullptr;  // C^T: n rows of (element node, weight)
  const int* trow = nullptr;
  const double* tval64 = nullptr;
  const float* tval32 = nullptr;
  const double* kref64 = nullptr;
  const float* kref32 = nullptr;
  const double* mref64 = nullptr;
  const float* mref32 = nullptr;
  const double* dinv64 = nullptr;
  const float* dinv32 = nullptr;
  // from the next coarser level: P (n rows) and P^T (coarse rows)
  const int* pptr = nullptr;
  const int* pcol = nullptr;
  const double* pval64 = nullptr;
  const float* pval32 = nullptr;
  const int* rptr = nullptr;
  const int* rcol = nullptr;
  const double* rval64 = nullptr;
  const float* rval32 = nullptr;
};

// Same epilogues as ApplyArgs; ye is scratch of E m values of the kernel precision.
struct OctApply {
  const void* x;
  void* out;
  const void* b;
  const void* xp;
  double c1, c2;
  Epi epi;
  void* ye;
};

hipError_t launch_oct_apply(const OctLevelDev& L, bool fp32, bool mass, const OctApply& a, hipStream_t s);
// uf += P ec;  rc = P^T rf (nc coarse DoFs)
hipError_t launch_oct_prolong(const OctLevelDev& fine, bool fp32, const void* ec, void* uf, hipStream_t s);
hipError_t launch_oct_restrict(const OctLevelDev& fine, int64_t nc, bool fp32, const void* rf, void* rc,
                               hipStream_t s);
// out = c d .* in (in null: out = c d; d null: d = 1), d an FP64 vector; in may alias out
hipError_t launch_vec_scale(bool fp32, int64_t n, const double* d, double c, const void* in, void* out,
                            hipStream_t s);

// uf += P ec (coarse Nc^3 -> fine (2Nc)^3) and rc = P^T rf, as three one-axis
// passes through the temporaries t1 (>= Nf^3/2 values) and t2 (>= Nf^3/4).
hipError_t launch_prolong(const TransferTab& tab, bool fp32, const void* ec, void* t1, void* t2, void* uf, int Nc,
                          hipStream_t s, bool fused = true);
hipError_t launch_restrict(const TransferTab& tab, bool fp32, const void* rf, void* t1, void* t2, void* rc, int Nc,
                           hipStream_t s, bool fused = true);
// fused: one kernel for the three axes (bit-identical to the axis passes), q <= 2:
// the prolongation from coarse levels of 2q <= Nc <= 256 nodes a side, the
// restriction onto those of 64 <= Nc <= 256; prime_transfer_shapes queries their
// occupancy once per level size, before any graph capture
void prime_transfer_shapes(int q, int Nc);
bool prolong_fusable(int q, int Nc);
bool restrict_fusable(int q, int Nc);

// out = c * tab[class(i)] * in  (class table of length q^3; in may be null -> 1)
hipError_t launch_class_scale(bool fp32, int q, int N, const double* tab, double c, const void* in, void* out,
                              hipStream_t s);

// Reductions: partial sums per block in FP64 into `part` (length >= kRedBlocks),
// then one block adds them in a fixed order into *dst (device).
constexpr int kRedBlocks = 1024;
hipError_t launch_dot(bool fp32, int64_t n, const void* x, const void* y, double* part, double* dst,
                      hipStream_t s);
hipError_t launch_sum(bool fp32, int64_t n, const void* x, double* part, double* dst, hipStream_t s);
// The dot of launch_dot with its partials in a static device array instead of `part`:
// kNoallocPartials FP64 values (8 KiB) per device.  noalloc_scratch_init(device), with that
// device current, looks the array's device address up once (at context setup);
// launch_dot_noalloc then allocates nothing.  Concurrent calls on one device share the
// array and race.
constexpr int kNoallocPartials = kRedBlocks;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch_init(int device);
hipError_t launch_dot_noalloc(int device, bool fp32, int64_t n, const void* x, const void* y, double* dst,
                              hipStream_t s);
// Fused Krylov reductions (part needs 3 * kRedBlocks doubles; results go to scalar slots of sc):
//   dot2:        sc[dxy] = x.y, sc[dxz] = x.z
//   axpy2_sums:  u += a p, r -= a w (a = sc[inum] / sc[iden]); sc[dsum] = sum r, sc[dsq] = r.r
//   sums3:       sc[dz] = sum z, sc[dzy] = z.y, sc[dy] = sum y
//   combine:     sc[dst] = sc[a] - sc[b] sc[c] scale (one thread)
//   xpby_shift:  p = (z - sc[imean] scale) + (sgn sc[inum] / sc[iden]) p
//   sq2:         sc[dx] = x.x, sc[dy] = y.y
hipError_t launch_sq2(bool fp32, int64_t n, const void* x, const void* y, double* part, double* sc, int dx, int dy,
                      hipStream_t s);
hipError_t launch_dot2(bool fp32, int64_t n, const void* x, const void* y, const void* z, double* part, double* sc,
                       int dxy, int dxz, hipStream_t s);
hipError_t launch_axpy2_sums(bool fp32, int64_t n, double* sc, int inum, int iden, void* u, const void* p, void* r,
                             const void* w, double* part, int dsum, int dsq, hipStream_t s);
hipError_t launch_sums3(bool fp32, int64_t n, const void* z, const void* y, double* part, double* sc, int dz,
                        int dzy, int dy, hipStream_t s);
hipError_t launch_combine(double* sc, int dst, int a, int b, int c, double scale, hipStream_t s);
hipError_t launch_xpby_shift(bool fp32, int64_t n, const double* sc, int inum, int iden, double sgn, int imean,
                             double scale, const void* z, void* p, hipStream_t s);
// sum_i tab[class(i)] x_i (the integral of the FE function on a uniform level);
// needs N^2 partials in `part` (capacity part_cap).
hipError_t launch_class_dot(bool fp32, int q, int N, const double* tab, const void* x, double* part,
                            int64_t part_cap, double* dst, hipStream_t s);

// Vector updates whose coefficients live in device memory (no host sync).
//  axpy2:   u += a p ; r -= a w        with a = sc[i_num] / sc[i_den]
//  xpby:    p = z + b p                with b = sgn * sc[i_num] / sc[i_den]
//  shift:   v -= sc[i] * scale         (projection: scale = 1/n)
hipError_t launch_axpy2(bool fp32, int64_t n, const double* sc, int i_num, int i_den, void* u, const void* p,
                        void* r, const void* w, hipStream_t s);
hipError_t launch_xpby(bool fp32, int64_t n, const double* sc, int i_num, int i_den, double sgn, const void* z,
                       void* p, hipStream_t s);
hipError_t launch_shift(bool fp32, int64_t n, const double* sc, int i, double scale, void* v, hipStream_t s);
// FP64 Krylov vectors around FP32 cycles: the (sum z, z.y, sum y) reductions and the
// p = (z - mean) + beta p update reading the FP32 cycle output z directly
hipError_t launch_sums3_mixed(int64_t n, const float* z, const double* y, double* part, double* sc, int dz, int dzy,
                              int dy, hipStream_t s);
// (sum z, z.w, sum w, z.r) -> sc[dz], sc[dzw], sc[dw], sc[dzr]
hipError_t launch_sums4_mixed(int64_t n, const float* z, const double* w, const double* r, double* part, double* sc,
                              int dz, int dzw, int dw, int dzr, hipStream_t s);
hipError_t launch_xpby_shift_mixed(int64_t n, const double* sc, int inum, int iden, double sgn, int imean,
                                   double scale, const float* z, double* p, hipStream_t s);
// r = src - sc[i] scale and r32 = float(r) in one pass (src may be r), with sc[dsq] =
// ||r||^2 (bits of a dot(r, r) after the shift) and sc[dsum] = sum of the shifted r
hipError_t launch_shift_cast_sq(int64_t n, double* sc, int i, double scale, const double* src, double* r, float* r32,
                                double* part, int dsq, int dsum, hipStream_t s);
// u = 0 and, of b, sc[dsum] = sum b and sc[dsq] = b . b in one pass
hipError_t launch_zero_sums(int64_t n, const double* b, double* u, double* part, double* sc, int dsum, int dsq,
                            hipStream_t s);
// (x.y, x.z, sum y) -> sc[dxy], sc[dxz], sc[dy]
hipError_t launch_dot2_sumy(int64_t n, const double* x, const double* y, const double* z, double* part, double* sc,
                            int dxy, int dxz, int dy, hipStream_t s);
// alpha = sc[inum] / sc[iden]; u += alpha p; r <- r - alpha w - m with the predicted mean
// m = (sc[irs] - alpha sc[iws]) scale; r32 = float(r); then sc[irs] = sum r, sc[dsq] = r.r
hipError_t launch_axpy2_cast(int64_t n, double* sc, int inum, int iden, int irs, int iws, double scale, double* u,
                             const double* p, double* r, const double* w, float* r32, double* part, int dsq,
                             hipStream_t s);
// p = double(z) - sc[i] scale (first direction from an FP32 cycle output)
hipError_t launch_shift_f2d(int64_t n, const double* sc, int i, double scale, const float* z, double* p,
                            hipStream_t s);

// y += a x with a host scalar; v_i += c tab[class(i)].
hipError_t launch_axpy(bool fp32, int64_t n, double a, const void* x, void* y, hipStream_t s);
hipError_t launch_class_axpy(bool fp32, int q, int N, const double* tab, double c, void* v, hipStream_t s);
// out_i = 2 U_i - 1 with U_i the i-th uniform double of the SplitMix64 stream `key`.
hipError_t launch_splitmix_start(uint64_t key, int64_t n, double* out, hipStream_t s);

// Precision conversions: f64 -> f32 and f32 -> f64 copies, and u64 += c32.
hipError_t launch_cast_d2f(int64_t n, const double* in, float* out, hipStream_t s);
hipError_t launch_cast_f2d(int64_t n, const float* in, double* out, hipStream_t s);
hipError_t launch_add_f2d(int64_t n, const float* c, double* u, hipStream_t s);
hipError_t launch_fill_zero(bool fp32, int64_t n, void* v, hipStream_t s);
hipError_t launch_copy(bool fp32, int64_t n, const void* in, void* out, hipStream_t s);

// *dst = sum of `count` FP64 partials, in a fixed order: one block, or for long runs
// a first pass over chunks of 64 into part[count ..] when part_cap has room for it.
hipError_t launch_sum_partials(const double* part, int64_t count, int64_t part_cap, double* dst, hipStream_t s);

// ---------------------------------------------------------------------------
// Learned smoother (gmg_net.hip): device state of one net.  Master weights w
// and Adam moments m, v are FP32 in the flat layout W1[co][t], W2[co][ci][t],
// W3[ci][t] (7776 values); w1q, w3q hold the BF16-rounded layer-1/3 weights
// tap-major as FP32; w2f / w2b are the BF16 A operands of the forward and
// backward-data layer-2 MFMA passes.
struct NetDev {
  float* w = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* w1q = nullptr;
  uint16_t* w2f = nullptr;
  uint16_t* w2b = nullptr;
  float* w3q = nullptr;
  // lane-ordered MFMA operands (16 bytes per entry): layer 2 forward and backward-data (15 x 64
  // each), layer 1 (2 x 64), layer 3 (2 x 64)
  void* w2fl = nullptr;
  void* w2bl = nullptr;
  void* w1l = nullptr;
  void* w3l = nullptr;  // layer 3 (2 x 64)
};
constexpr int kNetWeights = 7776;
// bytes of the forward cache (BF16 input + two 16-channel BF16 activations)
int64_t net_cache_bytes(int N);
// FP32 scratch values needed by the weight-gradient reductions
int64_t net_partial_floats(int N);
hipError_t launch_net_pack(const float* w, NetDev& d, hipStream_t s);
// cache.x_in = bf16(D^-1 r / s), s = RMS(D^-1 r) written to *ssum as a sum of squares
// (dinv == null: x_in = bf16(r), ssum unused); part needs N^2 doubles (part_cap of them
// are allocated; with N^2 + N^2/64 the partials are folded in two passes).  N a multiple of
// 4, r and cache 16-byte aligned (else hipErrorInvalidValue).
hipError_t launch_net_input(const float* r, const double* dinv, int q, const double* ssum, double* part,
                            int64_t part_cap, int N, void* cache, hipStream_t s);
// y = N(x_in) (mode 0) or y += s N(x_in) with s = sqrt(*ssum / N^3) (mode 1).
// The cache receives a2 always and a1 only with keep_a1 (what the backward pass reads).
hipError_t launch_net_forward(const NetDev& d, int N, void* cache, int mode, const double* ssum, float* y,
                              hipStream_t s, bool keep_a1 = true);
// gw += d(sum gy . y)/dw; gin = d(sum gy . y)/dx_in when non-null.  g1g2: 64 bytes per voxel.
hipError_t launch_net_backward(const NetDev& d, int N, const void* cache, const float* gy, void* g1g2, float* part,
                               float* gw, float* gin, hipStream_t s);
hipError_t launch_adam(NetDev& d, const float* gw, float lr, int64_t step, hipStream_t s);
// et = s y, s = sqrt(*ssum / n);   gy = -2 s scale d / (*er)
hipError_t launch_net_scale(const float* y, const double* ssum, int64_t n, float* et, hipStream_t s);
hipError_t launch_net_loss_gy(const float* d, const double* ssum, const double* er, double scale, int64_t n, float* gy,
                              hipStream_t s);

// Coarsest solve: x = Ainv (b - mean(b)), Ainv dense symmetric N0 x N0 (FP64),
// b and x of the kernel precision, arithmetic in FP64.
hipError_t launch_coarse(bool fp32, int n0, const double* ainv, const void* b, void* x, hipStream_t s);

// One-workgroup cycle on the uniform level of 16^3 nodes whose coarser
// neighbour is the coarsest level (8^3 nodes): the smoother steps are
// x' = x + c1[s] (x - x_prev) + c2[s] D^-1 (b - A x), npre of them from u = 0
// before the coarse-grid correction and npost after it.
constexpr int kTailMaxSteps = 24;
struct TailSteps {
  int npre, npost;
  double c1[kTailMaxSteps], c2[kTailMaxSteps];
};
bool tail_supported(int q, bool fp32, int N, int Nc, const TailSteps& st);
// u = pre-smoothed iterate from 0, bc = P^T (b - A u)   (u: 16^3, bc: 8^3)
hipError_t launch_tail_down(const OpTab& op, const TransferTab& xf, const TailSteps& st, bool fp32, const void* b,
                            void* u, void* bc, hipStream_t s);
// u += P ec, then the post-smoothing steps
hipError_t launch_tail_up(const OpTab& op, const TransferTab& xf, const TailSteps& st, bool fp32, const void* b,
                          void* u, const void* ec, hipStream_t s);

}  // namespace gmg
