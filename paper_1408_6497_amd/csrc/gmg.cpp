// Host orchestration and C ABI of the multigrid library.
//
// Setup (Section 2.3, "Setup"): mesh hierarchy of nested uniform periodic
// meshes (Section 2.3.1: every coarse element is the parent of 8 fine ones),
// operator tables and Jacobi diagonal, Lanczos estimate of lambda_max(D^-1 A)
// (Section 2.3.3), dense coarsest pseudo-inverse.  Solve: V-cycle of
// Algorithm 2.1 with Chebyshev-Jacobi smoothing, CG preconditioned by one
// V-cycle (Section 2.3), and FP64 iterative refinement around an FP32 flexible
// CG.  Every vector operation runs in the HIP kernels declared in
// gmg_kernels.h; the host only sequences launches and reads scalars back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <memory>
#include <vector>

#include "gmg.h"
#include "gmg_octree_host.h"
#include "gmg_kernels.h"
#include "gmg_setup_math.h"

using namespace gmg;

namespace {

constexpr int kNumScal = 64;
// device scalar slots
enum : int {
  S_PW = 0,   // p . w
  S_PR = 1,   // p . r
  S_RZ0 = 2,  // r . z (two slots, ping-pong)
  S_RZ1 = 3,
  S_ZW = 4,   // z . w
  S_SUM = 5,  // projection sum
  S_RR = 6,   // r . r
  S_TMP = 7,
  S_LRES = 8,   // ||r - A z||^2 of a cycle under test
  S_LRR = 9,    // ||r||^2 of that cycle's input
  S_ER = 10,    // e^T r        (training loss)
  S_ED = 11,    // e^T (r - A e~)
  S_TD = 12,    // e~^T (r - A e~)
  S_ZS = 13,    // sum z            (fused direction update)
  S_YS = 14,    // sum w or sum r   (fused direction update)
  S_ZWC = 15,   // (z - mean z) . w
  S_SSUM = 16,  // + level: sum of (D^-1 r)^2 of the learned correction on that level
  S_RS = 48,    // sum of the stored Krylov residual (FCG around FP32 cycles)
  S_WS = 49,    // sum of w = A p                      (the same)
  S_ZR = 50,    // z . r                                (the same)
  S_TR = 51,    // true residual's r . r and sum r      (the same, its final check)
  S_TS = 52,
};
// a hierarchy has at most 11 levels (n <= 512 uniform, leaf level <= 10 octree)
static_assert(S_SSUM + 32 <= S_RS && S_WS < kNumScal, "scalar slots overlap");

struct Level {
  int n = 0, N = 0;   // uniform: elements and lattice nodes per direction (0 on octree levels)
  // lattice nodes per direction of a level whose DoFs form a uniform lattice in lattice
  // order: every uniform level, and an octree level whose leaves all have one level (its
  // DoF numbering is the lattice order); 0 otherwise.  Such a level has the uniform
  // tables in `tab` (the learned correction reads its Jacobi diagonal by node class).
  int latN = 0;
  // orders without a specialised kernel (q = 3, 5, 6, 7, 8): the generic passes' device
  // tables, and the node-class tables (q^3 values) in device memory plus a host copy of
  // the diagonal
  bool gen = false;
  GenOp gstiff{}, gmass{};
  const double* gdiag = nullptr;
  const double* gdsqrt = nullptr;
  const double* gdinv_sqrt = nullptr;
  const double* gwint = nullptr;
  std::vector<double> gdiag_host;
  int64_t size = 0;
  LevelTables tab{};
  // octree levels: device arrays, and host copies of the leaves and DoF positions
  bool oct = false;
  OctLevelDev od{};
  double* diag64 = nullptr;
  double* dsqrt64 = nullptr;
  double* dinv_sqrt64 = nullptr;
  double* wint64 = nullptr;
  double w0w0 = 0.0;  // sum of the diagonal: ||D^1/2 1||^2
  std::vector<oct::Leaf> leaves;
  std::vector<int64_t> points;
  double lam = 0, alpha = 0, beta = 0;
  void* b[2] = {nullptr, nullptr};   // [0] FP64, [1] FP32
  void* u[2] = {nullptr, nullptr};
  void* xp[2] = {nullptr, nullptr};
};

}  // namespace

struct gmg_ctx {
  int q = 0, L = 0;
  int device = 0;                // the HIP device current at gmg_setup
  gmg_options opt{};
  hipStream_t user = nullptr;    // the caller's stream (gmg_setup argument)
  hipStream_t stream = nullptr;  // the library's own work stream, ordered with `user` by events
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // captured finest V-cycles: [0] FP64 on (kr0, kz0), [1] FP32 on (kr1, kz1),
  // [2] FP64 r -> FP32 V-cycle -> FP64 z on (kr0, kz0)
  // [3..6] the learned / plain test sequences of the learned cycle (see precondition)
  // captured launch sequences: 0-2 V-cycles, 3-6 learned cycles under test, 7-8 the
  // cycle plus direction update of FP64 flexible CG around FP32 cycles
  // 9-10: the direction updates after a learned cycle in that same loop
  static constexpr int kGraphKeys = 11;
  hipGraphExec_t vgraph[kGraphKeys] = {};
  bool graph_failed[kGraphKeys] = {};
  bool suppress_learned = false;
  std::vector<Level> lv;
  TransferTab xfer{};
  GenXfer gxfer{};             // transfer weights of an order without a specialised kernel
  bool gen = false;            // the order has no specialised kernels (every level is generic)
  void* gtmp[2][4] = {};       // the generic apply's four temporaries, per precision
  void* tA[2] = {nullptr, nullptr};
  void* tB[2] = {nullptr, nullptr};
  bool have_prec[2] = {false, false};
  double* ainv = nullptr;
  int n0 = 0;
  double* scal = nullptr;
  double* scal_host = nullptr;  // pinned host copy of scal (read back at each convergence test)
  hipEvent_t ev_copy = nullptr;  // marks the end of a read-back that later work overlaps
  std::unique_ptr<FftQ1> fft;    // plans and spectra of gmg_fft_solve (made on first use)
  std::unique_ptr<FftQ2> fft2;
  std::unique_ptr<FftQ4> fft4;
  hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;  // bracket each solve (gmg_info.t_solve)
  double* part = nullptr;
  int64_t part_cap = 0;
  // finest-level Krylov vectors per precision: r, z, p, w, c
  void* kr[2] = {nullptr, nullptr};
  void* kz[2] = {nullptr, nullptr};
  void* kp[2] = {nullptr, nullptr};
  void* kw[2] = {nullptr, nullptr};
  void* kc[2] = {nullptr, nullptr};
  void* bint = nullptr;  // FP64 load vector inside gmg_solve
  bool octree = false;
  void* oye[2] = {nullptr, nullptr};  // octree apply scratch: E m values of the largest level
  int64_t oye_size = 0;
  std::vector<void*> allocs;
  std::string err;
  double t_setup = 0.0;
  // launch timing (gmg_options.timing)
  struct Pending {
    hipEvent_t a, b;
    int level, kind, pi;
    int64_t n0 = 0, n1 = 0;  // kind < 0: a run of n0 + n1 smoother steps (kinds 2 and 3)
  };
  Pending run;            // open run of consecutive smoother steps (launch timing)
  bool run_open = false;
  bool group_runs = false;  // set while a smoothing phase launches its steps
  // learned smoother: one net per depth (depth 0 = finest level)
  std::vector<NetDev> nets;
  std::vector<char> net_set;
  std::vector<void*> lcache;      // per level: forward cache of the learned correction
  void* g1g2 = nullptr;           // backward scratch (64 bytes per voxel of the largest trained level)
  int64_t g1g2_bytes = 0;
  float* npart = nullptr;         // weight-gradient partials
  int64_t npart_floats = 0;
  double rho_plain = -1.0;        // most recent contraction of a plain FP32 cycle
  int64_t fallbacks = 0;
  std::vector<double> hist_res;   // last solve: Krylov residual norms, one per iteration
  std::vector<double> hist_cyc;   // last solve: (rho_learned, rho_reference, rho_plain) per cycle
  std::vector<hipEvent_t> ev_pool;
  std::vector<hipEvent_t> ev_all;
  std::vector<Pending> pending;
  std::vector<double> tsec;     // [level][kind][prec]
  std::vector<int64_t> tcount;
};

namespace {

inline int pidx(gmg_prec p) { return p == GMG_FP32 ? 1 : 0; }
inline size_t esize(int pi) { return pi ? sizeof(float) : sizeof(double); }

gmg_status fail(gmg_ctx* c, gmg_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(ctx, expr)                                                                     \
  do {                                                                                        \
    const hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                                     \
      return fail((ctx), GMG_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));      \
  } while (0)

#define STCHK(expr)                     \
  do {                                  \
    const gmg_status s_ = (expr);       \
    if (s_ != GMG_OK) return s_;        \
  } while (0)

gmg_status dalloc(gmg_ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  const hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(c, GMG_E_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  c->allocs.push_back(*p);
  return GMG_OK;
}

// Allocate every buffer of one precision (level vectors, transfer temporaries,
// Krylov vectors) on first use.
gmg_status ensure_prec(gmg_ctx* c, int pi) {
  if (c->have_prec[pi]) return GMG_OK;
  const size_t es = esize(pi);
  for (auto& L : c->lv) {
    STCHK(dalloc(c, &L.b[pi], L.size * es));
    STCHK(dalloc(c, &L.u[pi], L.size * es));
    STCHK(dalloc(c, &L.xp[pi], L.size * es));
  }
  const int64_t nf = c->lv.back().size;
  STCHK(dalloc(c, &c->tA[pi], (nf / 2 + 1) * es));
  STCHK(dalloc(c, &c->tB[pi], (nf / 4 + 1) * es));
  STCHK(dalloc(c, &c->kr[pi], nf * es));
  STCHK(dalloc(c, &c->kz[pi], nf * es));
  STCHK(dalloc(c, &c->kp[pi], nf * es));
  STCHK(dalloc(c, &c->kw[pi], nf * es));
  STCHK(dalloc(c, &c->kc[pi], nf * es));
  if (c->gen)
    for (int t = 0; t < 4; ++t) STCHK(dalloc(c, &c->gtmp[pi][t], nf * es));
  c->have_prec[pi] = true;
  return GMG_OK;
}

// launch-timing kinds (gmg_timing_get)
enum : int {
  K_APPLY = 0,
  K_RESIDUAL = 1,
  K_SMOOTH0 = 2,
  K_SMOOTH = 3,
  K_MASS = 4,
  K_RESTRICT = 5,
  K_PROLONG = 6,
  K_COARSE = 7,
  K_LEARNED = 8,
  K_SCALE = 9,    // first smoother step from a zero guess: x = c D^-1 b (no operator apply)
  K_SMOOTHZ = 10,  // first two Chebyshev steps from a zero guess in one pass
  K_TAIL = 11,     // one-workgroup cycle on the 16^3-node level (smoothing, residual, transfers)
};
constexpr int kKinds = 12;
inline int tslot(int level, int kind, int pi) { return (level * kKinds + kind) * 2 + pi; }

hipEvent_t take_event(gmg_ctx* c) {
  if (c->ev_pool.empty()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_all.push_back(e);
    return e;
  }
  hipEvent_t e = c->ev_pool.back();
  c->ev_pool.pop_back();
  return e;
}

// Fold every completed event pair into the per-(level, kind, prec) sums.
gmg_status drain_timing(gmg_ctx* c) {
  if (c->pending.empty()) return GMG_OK;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (const auto& p : c->pending) {
    float ms = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, p.a, p.b));
    if (p.kind < 0) {
      // a run of smoother steps: its time is split between the two step kinds in
      // proportion to their algorithmic traffic (3 and 4 values per DoF)
      const double w0 = 3.0 * static_cast<double>(p.n0), w1 = 4.0 * static_cast<double>(p.n1);
      const int s0 = tslot(p.level, K_SMOOTH0, p.pi), s1 = tslot(p.level, K_SMOOTH, p.pi);
      c->tsec[s0] += 1e-3 * ms * w0 / (w0 + w1);
      c->tsec[s1] += 1e-3 * ms * w1 / (w0 + w1);
      c->tcount[s0] += p.n0;
      c->tcount[s1] += p.n1;
    } else {
      const int s = tslot(p.level, p.kind, p.pi);
      c->tsec[s] += 1e-3 * ms;
      c->tcount[s] += 1;
    }
    c->ev_pool.push_back(p.a);
    c->ev_pool.push_back(p.b);
  }
  c->pending.clear();
  return GMG_OK;
}

// Close the open run of smoother steps: its end event goes right after its last launch.
gmg_status close_run(gmg_ctx* c) {
  if (!c->run_open) return GMG_OK;
  c->run_open = false;
  HIPCHK(c, hipEventRecord(c->run.b, c->stream));
  c->pending.push_back(c->run);
  if (c->pending.size() > 4096) STCHK(drain_timing(c));
  return GMG_OK;
}

// With launch timing on, bracket the work `body` enqueues with HIP events, filed under
// (level, kind, precision); otherwise just run it.
template <class F>
gmg_status timed(gmg_ctx* c, int l, int kind, int pi, F&& body) {
  if (!c->opt.timing) return body();
  STCHK(close_run(c));
  hipEvent_t ea = take_event(c), eb = take_event(c);
  if (!ea || !eb) return fail(c, GMG_E_HIP, "hipEventCreate failed");
  HIPCHK(c, hipEventRecord(ea, c->stream));
  const gmg_status st = body();
  HIPCHK(c, hipEventRecord(eb, c->stream));
  c->pending.push_back({ea, eb, l, kind, pi});
  if (c->pending.size() > 4096) STCHK(drain_timing(c));
  return st;
}

// Seconds per phase over every level and precision since the last reset:
// smoother steps, transfers, coarsest solve, learned corrections.
void phase_totals(const gmg_ctx* c, double out[4]) {
  out[0] = out[1] = out[2] = out[3] = 0.0;
  for (int l = 0; l < c->L; ++l)
    for (int pi = 0; pi < 2; ++pi) {
      auto t = [&](int k) { return c->tsec[tslot(l, k, pi)]; };
      out[0] += t(K_SMOOTH0) + t(K_SMOOTH) + t(K_SCALE) + t(K_SMOOTHZ) + t(K_TAIL);
      out[1] += t(K_RESTRICT) + t(K_PROLONG);
      out[2] += t(K_COARSE);
      out[3] += t(K_LEARNED);
    }
}

gmg_status apply_op(gmg_ctx* c, int l, int pi, Epi epi, const void* x, void* out, const void* b, const void* xp,
                    double c1, double c2, bool mass = false, void* x1 = nullptr, double s0 = 0.0, int d0 = -1,
                    int d1 = -1) {
  const Level& L = c->lv[l];
  // the uniform kernel moves q consecutive values per vector access
  const uintptr_t al = static_cast<uintptr_t>((L.oct || L.gen) ? 1 : c->q) * esize(pi);
  for (const void* ptr : {x, static_cast<const void*>(out), b, xp, static_cast<const void*>(x1)})
    if (ptr && (reinterpret_cast<uintptr_t>(ptr) % al) != 0)
      return fail(c, GMG_E_ARG, "device buffer not aligned to q elements");
  if (L.oct && !c->oye[pi]) return fail(c, GMG_E_STATE, "octree scratch of this precision not allocated");
  ApplyArgs a{};
  a.N = L.N;
  a.n = L.n;
  a.x = x;
  a.out = out;
  a.b = b;
  a.xp = xp;
  a.c1 = c1;
  a.c2 = c2;
  a.epi = epi;
  a.x1 = x1;
  a.s0 = s0;
  a.mfma = c->opt.q4_mfma != 0;
  if (epi == Epi::ApplyDot || epi == Epi::ResidualSums || epi == Epi::ResidualNorms) {
    if (L.oct || L.gen || (pi != 0 && epi != Epi::ResidualNorms) || mass || d0 < 0 || d1 < 0 || L.N <= 32)
      return fail(c, GMG_E_ARG, "fused apply and dot unsupported here");
    a.part = c->part;
    a.part_cap = c->part_cap;
    a.sc = c->scal;
    a.d0 = d0;
    a.d1 = d1;
  }
  hipEvent_t ea = nullptr, eb = nullptr;
  // Inside a smoothing phase, consecutive plain smoother steps on one level are
  // timed as one run (one event pair around all of them), so that the events'
  // own dispatch time is not added to every launch.
  const bool in_run = c->opt.timing && c->group_runs && epi == Epi::Cheb && !mass;
  if (c->opt.timing && !in_run) {
    STCHK(close_run(c));
    ea = take_event(c);
    eb = take_event(c);
    if (!ea || !eb) return fail(c, GMG_E_HIP, "hipEventCreate failed");
    HIPCHK(c, hipEventRecord(ea, c->stream));
  }
  if (in_run && c->run_open && (c->run.level != l || c->run.pi != pi)) STCHK(close_run(c));
  if (in_run && !c->run_open) {
    ea = take_event(c);
    eb = take_event(c);
    if (!ea || !eb) return fail(c, GMG_E_HIP, "hipEventCreate failed");
    HIPCHK(c, hipEventRecord(ea, c->stream));
    c->run = gmg_ctx::Pending{ea, eb, l, -1, pi, 0, 0};
    c->run_open = true;
  }
  if (L.oct) {
    const OctApply oa{x, out, b, xp, c1, c2, epi, c->oye[pi]};
    HIPCHK(c, launch_oct_apply(L.od, pi == 1, mass, oa, c->stream));
  } else if (L.gen) {
    if (!c->gtmp[pi][0]) return fail(c, GMG_E_STATE, "generic apply temporaries of this precision not allocated");
    HIPCHK(c, launch_gen_apply(mass ? L.gmass : L.gstiff, pi == 1, a, c->gtmp[pi], c->stream));
  } else {
    HIPCHK(c, launch_apply(mass ? L.tab.mass : L.tab.stiff, pi == 1, a, c->stream));
  }
  if (in_run) {
    if (xp != nullptr && c1 != 0.0) ++c->run.n1;
    else ++c->run.n0;
  } else if (c->opt.timing) {
    HIPCHK(c, hipEventRecord(eb, c->stream));
    int kind = K_APPLY;
    if (mass) kind = K_MASS;
    else if (epi == Epi::Residual || epi == Epi::ResidualNorms) kind = K_RESIDUAL;
    else if (epi == Epi::Cheb) kind = (xp != nullptr && c1 != 0.0) ? K_SMOOTH : K_SMOOTH0;
    else if (epi == Epi::ChebZero) kind = K_SMOOTHZ;
    c->pending.push_back({ea, eb, l, kind, pi});
    if (c->pending.size() > 4096) STCHK(drain_timing(c));
  }
  return GMG_OK;
}

// The scalars go through a pinned buffer: a copy into pageable memory would be staged.
gmg_status read_scalars(gmg_ctx* c, double* host, int count) {
  HIPCHK(c, hipMemcpyAsync(c->scal_host, c->scal, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::memcpy(host, c->scal_host, sizeof(double) * count);
  return GMG_OK;
}

// The same read-back in two halves: scalars_async enqueues the copy of the scalars
// as they stand at this point of the work stream and an event after it, so that
// work enqueued next follows the copy at once while the host waits in
// scalars_wait (one stream: no cross-queue synchronisation, and the work after the
// copy may overwrite the slots it copied).
gmg_status scalars_async(gmg_ctx* c, int count) {
  HIPCHK(c, hipMemcpyAsync(c->scal_host, c->scal, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipEventRecord(c->ev_copy, c->stream));
  return GMG_OK;
}

gmg_status scalars_wait(gmg_ctx* c, double* host, int count) {
  HIPCHK(c, hipEventSynchronize(c->ev_copy));
  std::memcpy(host, c->scal_host, sizeof(double) * count);
  return GMG_OK;
}

// v <- v - mean(v)
gmg_status project(gmg_ctx* c, int pi, int64_t n, void* v) {
  HIPCHK(c, launch_sum(pi == 1, n, v, c->part, c->scal + S_SUM, c->stream));
  HIPCHK(c, launch_shift(pi == 1, n, c->scal, S_SUM, 1.0 / static_cast<double>(n), v, c->stream));
  return GMG_OK;
}

// out = w D^-1 b on one level
hipError_t dinv_scale(gmg_ctx* c, const Level& L, bool f32, double w, const void* b, void* out) {
  if (L.oct) return launch_vec_scale(f32, L.size, L.od.dinv64, w, b, out, c->stream);
  if (L.gen) return launch_gclass_scale(f32, c->q, L.N, L.gstiff.dinv64, w, b, out, c->stream);
  return launch_class_scale(f32, c->q, L.N, L.tab.stiff.dinv, w, b, out, c->stream);
}

// u <- S^nu(u; b) on level l.  zero_init: u is taken as 0 on entry (not read).
gmg_status smooth(gmg_ctx* c, int l, int pi, const void* b, void* u, int nu, bool zero_init) {
  Level& L = c->lv[l];
  const bool f32 = pi == 1;
  if (nu <= 0) {
    if (zero_init) HIPCHK(c, launch_fill_zero(f32, L.size, u, c->stream));
    return GMG_OK;
  }
  void* bufs[2] = {u, L.xp[pi]};
  int cur = 0;
  bool prev_zero = false;
  bool x_zero = zero_init;
  // launch timing: the plain steps of this phase are timed in runs (closed below)
  struct RunScope {
    gmg_ctx* c;
    explicit RunScope(gmg_ctx* cc) : c(cc) { c->group_runs = true; }
    ~RunScope() { c->group_runs = false; }
  } scope(c);
  if (c->opt.smoother == 1) {
    const double w = c->opt.jacobi_omega;
    for (int s = 0; s < nu; ++s) {
      if (x_zero) {
        STCHK(timed(c, l, K_SCALE, pi, [&]() -> gmg_status {
          HIPCHK(c, dinv_scale(c, L, f32, w, b, bufs[1 - cur]));
          return GMG_OK;
        }));
        x_zero = false;
      } else {
        STCHK(apply_op(c, l, pi, Epi::Cheb, bufs[cur], bufs[1 - cur], b, nullptr, 0.0, w));
      }
      cur ^= 1;
    }
  } else {
    const double theta = 0.5 * (L.beta + L.alpha);
    const double delta = 0.5 * (L.beta - L.alpha);
    const double sigma = theta / delta;
    const int deg = c->opt.cheb_degree;
    // from a zero guess on a uniform level the scaling x_1 = D^-1 b / theta is not a
    // pass of its own: the next step forms x_1 from b as it loads it (Epi::ChebZero)
    const bool fuse_zero = !L.oct && !L.gen && deg >= 2;
    double s0 = 0.0;
    for (int app = 0; app < nu; ++app) {
      double rho = 1.0 / sigma;
      for (int j = 0; j < deg; ++j) {
        double c1 = 0.0, c2 = 1.0 / theta;
        if (j > 0) {
          const double rho_new = 1.0 / (2.0 * sigma - rho);
          c1 = rho_new * rho;
          c2 = 2.0 * rho_new / delta;
          rho = rho_new;
        }
        if (x_zero && fuse_zero) {
          s0 = c2;  // x_1 = s0 D^-1 b, formed by the next launch into bufs[1 - cur]
          x_zero = false;
          prev_zero = true;
        } else if (prev_zero && s0 != 0.0) {
          // x_2 = x_1 + c1 x_1 + c2 D^-1 (b - A x_1), storing x_1 where the scaling would have
          STCHK(apply_op(c, l, pi, Epi::ChebZero, b, bufs[1 - cur], b, nullptr, c1, c2, false, bufs[cur], s0));
          s0 = 0.0;
          prev_zero = false;
        } else if (x_zero) {
          // x_1 = x_0 + D^-1 (b - A x_0) / theta with x_0 = 0
          STCHK(timed(c, l, K_SCALE, pi, [&]() -> gmg_status {
            HIPCHK(c, dinv_scale(c, L, f32, c2, b, bufs[1 - cur]));
            return GMG_OK;
          }));
          x_zero = false;
          prev_zero = true;
        } else {
          const void* xpp = (c1 != 0.0 && !prev_zero) ? bufs[1 - cur] : nullptr;
          STCHK(apply_op(c, l, pi, Epi::Cheb, bufs[cur], bufs[1 - cur], b, xpp, c1, c2));
          prev_zero = false;
        }
        cur ^= 1;
      }
    }
  }
  STCHK(close_run(c));
  if (bufs[cur] != u) HIPCHK(c, launch_copy(f32, L.size, bufs[cur], u, c->stream));
  return GMG_OK;
}

// rc = P^T rf, fine level l -> l-1
gmg_status restrict_level(gmg_ctx* c, int l, int pi, const void* rf, void* rc) {
  const int Nc = c->lv[l - 1].N;
  const bool f32 = pi == 1;
  return timed(c, l, K_RESTRICT, pi, [&]() -> gmg_status {
    if (c->lv[l].oct) HIPCHK(c, launch_oct_restrict(c->lv[l].od, c->lv[l - 1].size, f32, rf, rc, c->stream));
    else if (c->lv[l].gen) HIPCHK(c, launch_gen_restrict(c->gxfer, f32, rf, c->tA[pi], c->tB[pi], rc, Nc, c->stream));
    else
      HIPCHK(c, launch_restrict(c->xfer, f32, rf, c->tA[pi], c->tB[pi], rc, Nc, c->stream, !c->opt.no_fused_transfer));
    return GMG_OK;
  });
}

// uf += P ec, level l-1 -> l
gmg_status prolong_level(gmg_ctx* c, int l, int pi, const void* ec, void* uf) {
  const int Nc = c->lv[l - 1].N;
  const bool f32 = pi == 1;
  return timed(c, l, K_PROLONG, pi, [&]() -> gmg_status {
    if (c->lv[l].oct) HIPCHK(c, launch_oct_prolong(c->lv[l].od, f32, ec, uf, c->stream));
    else if (c->lv[l].gen) HIPCHK(c, launch_gen_prolong(c->gxfer, f32, ec, c->tB[pi], c->tA[pi], uf, Nc, c->stream));
    else
      HIPCHK(c, launch_prolong(c->xfer, f32, ec, c->tB[pi], c->tA[pi], uf, Nc, c->stream, !c->opt.no_fused_transfer));
    return GMG_OK;
  });
}

gmg_status coarse_solve(gmg_ctx* c, int pi, const void* b, void* x) {
  return timed(c, 0, K_COARSE, pi, [&]() -> gmg_status {
    HIPCHK(c, launch_coarse(pi == 1, c->n0, c->ainv, b, x, c->stream));
    return GMG_OK;
  });
}

// Net used at depth d: its own if set, else the deepest (largest depth) net that is set.
int net_for_depth(const gmg_ctx* c, int d) {
  if (d >= 0 && d < static_cast<int>(c->net_set.size()) && c->net_set[d]) return d;
  for (int k = static_cast<int>(c->net_set.size()) - 1; k >= 0; --k)
    if (c->net_set[k]) return k;
  return -1;
}

bool learned_on_level(const gmg_ctx* c, int l, int pi) {
  const int d = c->L - 1 - l;
  if (c->opt.learned_depths > 0 && d >= c->opt.learned_depths) return false;
  if (d < c->opt.learned_min_depth) return false;
  // the lattice convolution needs a level whose DoFs form a uniform lattice (every uniform
  // level; of an octree hierarchy, the levels whose leaves all have one level)
  return c->opt.use_learned && !c->suppress_learned && pi == 1 && l > 0 && c->lv[l].latN >= 16 &&
         net_for_depth(c, d) >= 0;
}

gmg_status ensure_lcache(gmg_ctx* c, int l) {
  if (c->lcache[l]) return GMG_OK;
  return dalloc(c, &c->lcache[l], static_cast<size_t>(net_cache_bytes(c->lv[l].latN)));
}

// u <- u + s N_d(D^-1 (b - A u) / s) on level l (FP32), s = RMS(D^-1 (b - A u)).
gmg_status learned_correction(gmg_ctx* c, int l, const void* b, void* u) {
  Level& L = c->lv[l];
  const int d = net_for_depth(c, c->L - 1 - l);
  STCHK(ensure_lcache(c, l));
  return timed(c, l, K_LEARNED, 1, [&]() -> gmg_status {
    STCHK(apply_op(c, l, 1, Epi::Residual, u, L.xp[1], b, nullptr, 0, 0));
    HIPCHK(c, launch_net_input(static_cast<const float*>(L.xp[1]), L.tab.stiff.dinv, c->q, c->scal + S_SSUM + l,
                               c->part, c->part_cap, L.latN, c->lcache[l], c->stream));
    HIPCHK(c, launch_net_forward(c->nets[d], L.latN, c->lcache[l], 1, c->scal + S_SSUM + l, static_cast<float*>(u),
                                 c->stream, false));
    return GMG_OK;
  });
}

// Smoother coefficients of one smoothing phase on level l (the recurrence of
// smooth(): Chebyshev steps j = 0 .. degree-1 per application, or Jacobi steps).
void phase_steps(const gmg_ctx* c, const Level& L, int nu, int* count, double* c1, double* c2) {
  int k = *count;
  if (c->opt.smoother == 1) {
    for (int s = 0; s < nu; ++s, ++k) {
      c1[k] = 0.0;
      c2[k] = c->opt.jacobi_omega;
    }
  } else {
    const double theta = 0.5 * (L.beta + L.alpha);
    const double delta = 0.5 * (L.beta - L.alpha);
    const double sigma = theta / delta;
    for (int app = 0; app < nu; ++app) {
      double rho = 1.0 / sigma;
      for (int j = 0; j < c->opt.cheb_degree; ++j, ++k) {
        c1[k] = 0.0;
        c2[k] = 1.0 / theta;
        if (j > 0) {
          const double rho_new = 1.0 / (2.0 * sigma - rho);
          c1[k] = rho_new * rho;
          c2[k] = 2.0 * rho_new / delta;
          rho = rho_new;
        }
      }
    }
  }
  *count = k;
}

// The level of 16^3 nodes next to the coarsest runs its whole cycle in two
// one-workgroup launches around the coarsest solve (uniform levels, plain smoother).
bool fused_tail(const gmg_ctx* c, int l, int pi, TailSteps* st) {
  if (l != 1 || c->opt.no_fused_tail || c->lv[l].oct || c->lv[l].gen || learned_on_level(c, l, pi)) return false;
  const int deg = c->opt.smoother == 1 ? 1 : c->opt.cheb_degree;
  if (c->opt.nu_pre < 0 || c->opt.nu_post < 0 || deg < 1 ||
      static_cast<int64_t>(c->opt.nu_pre + c->opt.nu_post) * deg > kTailMaxSteps)
    return false;
  int k = 0;
  phase_steps(c, c->lv[l], c->opt.nu_pre, &k, st->c1, st->c2);
  st->npre = k;
  phase_steps(c, c->lv[l], c->opt.nu_post, &k, st->c1, st->c2);
  st->npost = k - st->npre;
  return tail_supported(c->q, pi == 1, c->lv[l].N, c->lv[0].N, *st);
}

// Algorithm 2.1 on level l with zero initial guess: u = V_l b.
gmg_status vcycle_level(gmg_ctx* c, int l, int pi, const void* b, void* u) {
  if (l == 0) return coarse_solve(c, pi, b, u);
  Level& L = c->lv[l];
  Level& C = c->lv[l - 1];
  TailSteps st{};
  if (fused_tail(c, l, pi, &st)) {
    const bool f32 = pi == 1;
    STCHK(timed(c, l, K_TAIL, pi, [&]() -> gmg_status {
      HIPCHK(c, launch_tail_down(L.tab.stiff, c->xfer, st, f32, b, u, C.b[pi], c->stream));
      return GMG_OK;
    }));
    STCHK(coarse_solve(c, pi, C.b[pi], C.u[pi]));
    STCHK(timed(c, l, K_TAIL, pi, [&]() -> gmg_status {
      HIPCHK(c, launch_tail_up(L.tab.stiff, c->xfer, st, f32, b, u, C.u[pi], c->stream));
      return GMG_OK;
    }));
    return GMG_OK;
  }
  // learned cycle: in each smoothing phase the last polynomial application is
  // replaced by one learned correction
  const bool lrn = learned_on_level(c, l, pi);
  const int nu_pre = lrn ? c->opt.nu_pre - 1 : c->opt.nu_pre;
  const int nu_post = lrn ? c->opt.nu_post - 1 : c->opt.nu_post;
  STCHK(smooth(c, l, pi, b, u, nu_pre, true));                                    // pre-smooth
  if (lrn) STCHK(learned_correction(c, l, b, u));
  STCHK(apply_op(c, l, pi, Epi::Residual, u, L.xp[pi], b, nullptr, 0, 0));       // residual
  STCHK(restrict_level(c, l, pi, L.xp[pi], C.b[pi]));                             // restrict
  STCHK(vcycle_level(c, l - 1, pi, C.b[pi], C.u[pi]));                            // recurse
  STCHK(prolong_level(c, l, pi, C.u[pi], u));                                     // correct
  STCHK(smooth(c, l, pi, b, u, nu_post, false));                                  // post-smooth
  if (lrn) STCHK(learned_correction(c, l, b, u));
  return GMG_OK;
}

// Every API call that enqueues work runs it on the library stream, after the
// work already queued on the caller's stream, and makes the caller's stream
// wait for it before returning.
template <class F>
gmg_status scoped(gmg_ctx* c, F&& body) {
  HIPCHK(c, hipEventRecord(c->ev_in, c->user));
  HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_in, 0));
  const gmg_status st = body();
  HIPCHK(c, hipEventRecord(c->ev_out, c->stream));
  HIPCHK(c, hipStreamWaitEvent(c->user, c->ev_out, 0));
  return st;
}

// z = V r on the finest level, in precision vpi, for Krylov vectors of
// precision pi (vpi = FP32 with pi = FP64 casts r down and z back up).  Inside
// the Krylov loops r and z are always the context's own vectors, so the
// sequence (a few dozen launches with fixed arguments) is captured once into a
// HIP graph and replayed.  With launch timing on, or if capture fails, it runs
// eagerly.
gmg_status vcycle_seq(gmg_ctx* c, int pi, int vpi, const void* r, void* z) {
  const int l = c->L - 1;
  if (pi == vpi) return vcycle_level(c, l, pi, r, z);
  const int64_t n = c->lv[l].size;
  HIPCHK(c, launch_cast_d2f(n, static_cast<const double*>(r), static_cast<float*>(c->kr[1]), c->stream));
  STCHK(vcycle_level(c, l, 1, c->kr[1], c->kz[1]));
  HIPCHK(c, launch_cast_f2d(n, static_cast<const float*>(c->kz[1]), static_cast<double*>(z), c->stream));
  return GMG_OK;
}

// Run a launch sequence with fixed arguments through a HIP graph captured on
// first use (eagerly with launch timing on, with no_graphs, or if capture fails).
template <class F>
gmg_status graph_run(gmg_ctx* c, int key, F&& seq) {
  if (c->opt.timing || c->opt.no_graphs || c->graph_failed[key]) return seq();
  if (!c->vgraph[key]) {
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    const gmg_status st = seq();
    const hipError_t e = hipStreamEndCapture(c->stream, &g);
    hipGraphExec_t ex = nullptr;
    if (st != GMG_OK || e != hipSuccess || !g || hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      c->graph_failed[key] = true;
      return seq();
    }
    (void)hipGraphDestroy(g);
    c->vgraph[key] = ex;
  }
  HIPCHK(c, hipGraphLaunch(c->vgraph[key], c->stream));
  return GMG_OK;
}

gmg_status run_vcycle(gmg_ctx* c, int pi, int vpi, const void* r, void* z) {
  const int key = (pi == vpi) ? pi : 2;
  if (r != c->kr[pi] || z != c->kz[pi]) return vcycle_seq(c, pi, vpi, r, z);
  return graph_run(c, key, [&] { return vcycle_seq(c, pi, vpi, r, z); });
}

// One FP32 cycle under test: z32 = V r32 (learned or plain), then
// ||r32 - A z32||^2 -> S_LRES and ||r32||^2 -> S_LRR.  r is the Krylov residual
// (FP64 when pi = 0: cast down first).  With keep_residual the residual r32 - A z32
// is left in the finest level's xp[1]; otherwise, on uniform levels of more than 32
// nodes, both norms come out of the residual's epilogue and it is not stored.
gmg_status test_cycle(gmg_ctx* c, int pi, const void* r, bool plain, bool keep_residual = false) {
  const int l = c->L - 1;
  const int64_t n = c->lv[l].size;
  void* r32 = c->kr[1];
  if (pi == 0) HIPCHK(c, launch_cast_d2f(n, static_cast<const double*>(r), static_cast<float*>(r32), c->stream));
  c->suppress_learned = plain;
  const gmg_status st = vcycle_level(c, l, 1, r32, c->kz[1]);
  c->suppress_learned = false;
  STCHK(st);
  const Level& L = c->lv[l];
  if (!keep_residual && !c->opt.no_fused_test_norms && !L.oct && !L.gen && L.N > 32) {
    // both norms in the residual's epilogue, the residual itself not stored
    return apply_op(c, l, 1, Epi::ResidualNorms, c->kz[1], nullptr, r32, nullptr, 0, 0, false, nullptr, 0.0, S_LRES,
                    S_LRR);
  }
  void* t = L.xp[1];
  STCHK(apply_op(c, l, 1, Epi::Residual, c->kz[1], t, r32, nullptr, 0, 0));
  HIPCHK(c, launch_sq2(true, n, t, r32, c->part, c->scal, S_LRES, S_LRR, c->stream));
  return GMG_OK;
}

// Contraction of the plain FP32 cycle, initialized by two plain cycles on a
// seeded mean-zero vector (SplitMix64 key seed + 7777).
gmg_status init_rho_plain(gmg_ctx* c) {
  const int l = c->L - 1;
  const int64_t n = c->lv[l].size;
  double hs[kNumScal];
  HIPCHK(c, launch_splitmix_start(c->opt.seed + 7777, n, static_cast<double*>(c->kc[0]), c->stream));
  STCHK(project(c, 0, n, c->kc[0]));
  double rho = 0.0;
  for (int k = 0; k < 2; ++k) {
    STCHK(test_cycle(c, 0, c->kc[0], true, true));
    STCHK(read_scalars(c, hs, kNumScal));
    rho = std::sqrt(hs[S_LRES] / hs[S_LRR]);
    // next input: the residual of this cycle, widened to FP64
    HIPCHK(c, launch_cast_f2d(n, static_cast<const float*>(c->lv[l].xp[1]), static_cast<double*>(c->kc[0]),
                              c->stream));
  }
  c->rho_plain = rho;
  return GMG_OK;
}

// Everything the learned cycles need before any graph capture: FP32 buffers,
// the forward caches of the levels that use a net, and the reference
// contraction of the plain cycle.
gmg_status prepare_learned(gmg_ctx* c) {
  if (!c->opt.use_learned || net_for_depth(c, 0) < 0) return GMG_OK;
  STCHK(ensure_prec(c, 1));
  for (int l = 1; l < c->L; ++l)
    if (learned_on_level(c, l, 1)) STCHK(ensure_lcache(c, l));
  if (c->rho_plain < 0.0) STCHK(init_rho_plain(c));
  return GMG_OK;
}

// z = preconditioner(r).  With the learned smoother active, one learned cycle is
// tried and kept if its contraction is no worse than the plain cycle's most
// recent one; otherwise the plain FP32 cycle is used (a fallback) and its
// contraction becomes the new reference.
// Is the finest-level cycle of precision vpi a learned one (with its per-cycle test)?
bool learned_precond(const gmg_ctx* c, int vpi) {
  return c->opt.use_learned && vpi == 1 && net_for_depth(c, 0) >= 0;
}

// The two halves of a learned preconditioner step: enqueue the learned cycle under test
// (z32 = V_L r, then ||r32 - A z32||^2 and ||r32||^2; reads nothing back), and read its
// contraction, run the plain cycle instead when it is worse (a fallback), and record the
// decision.  The mixed-precision flexible CG enqueues the first half behind the read-back
// of the residual norm and takes the second once the norm says the iteration goes on.
gmg_status learned_test_enqueue(gmg_ctx* c, int pi, int vpi, const void* r) {
  if (c->rho_plain < 0.0) return fail(c, GMG_E_STATE, "learned cycle used before prepare_learned");
  const int base = 3 + (pi == vpi ? 2 : 0);
  return graph_run(c, base, [&] { return test_cycle(c, pi, r, false); });
}

gmg_status learned_decide(gmg_ctx* c, int pi, int vpi, const void* r) {
  double hs[kNumScal];
  const int base = 3 + (pi == vpi ? 2 : 0);
  STCHK(read_scalars(c, hs, kNumScal));
  const double rho_l = std::sqrt(hs[S_LRES] / hs[S_LRR]);
  const double rho_ref = c->rho_plain;
  double rho_p = std::nan("");
  if (!(rho_l <= c->rho_plain)) {
    ++c->fallbacks;
    STCHK(graph_run(c, base + 1, [&] { return test_cycle(c, pi, r, true); }));
    STCHK(read_scalars(c, hs, kNumScal));
    c->rho_plain = rho_p = std::sqrt(hs[S_LRES] / hs[S_LRR]);
  }
  c->hist_cyc.insert(c->hist_cyc.end(), {rho_l, rho_ref, rho_p});
  return GMG_OK;
}

gmg_status precondition(gmg_ctx* c, int pi, int vpi, const void* r, void* z) {
  if (!learned_precond(c, vpi)) return run_vcycle(c, pi, vpi, r, z);
  const int l = c->L - 1;
  const int64_t n = c->lv[l].size;
  STCHK(learned_test_enqueue(c, pi, vpi, r));
  STCHK(learned_decide(c, pi, vpi, r));
  if (pi == 0) HIPCHK(c, launch_cast_f2d(n, static_cast<const float*>(c->kz[1]), static_cast<double*>(z), c->stream));
  else if (z != c->kz[1]) HIPCHK(c, launch_copy(true, n, c->kz[1], z, c->stream));
  return GMG_OK;
}

// Largest Ritz value of Lanczos on D^-1/2 A D^-1/2 (FP64, on the device).
gmg_status lanczos(gmg_ctx* c, int l, double* lam_out) {
  Level& L = c->lv[l];
  const int q = c->q;
  const int64_t n = L.size;
  void* v = L.b[0];
  void* vprev = L.u[0];
  void* w = L.xp[0];
  void* t = c->kr[0];
  const hipStream_t s = c->stream;
  const double ones[kMaxQ * kMaxQ * kMaxQ] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1,
                                              1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1,
                                              1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
  // the level's diagonal as a class table (uniform) or a vector (octree)
  auto scale = [&](const double* tab, const double* vec, const double* gtab, double a, const void* in, void* out) {
    if (L.oct) return launch_vec_scale(false, n, vec, a, in, out, s);
    if (L.gen) return launch_gclass_scale(false, q, L.N, gtab, a, in, out, s);
    return launch_class_scale(false, q, L.N, tab, a, in, out, s);
  };
  HIPCHK(c, launch_splitmix_start(c->opt.seed + static_cast<uint64_t>(l), n, static_cast<double*>(v), s));
  // project out the null vector D^1/2 1 of the scaled operator
  double w0w0 = 0.0;
  if (L.oct) {
    w0w0 = L.w0w0;
    HIPCHK(c, launch_dot(false, n, L.dsqrt64, v, c->part, c->scal + S_TMP, s));
  } else if (L.gen) {
    const int64_t per_class = n / (q * q * q);
    for (int i = 0; i < q * q * q; ++i) w0w0 += L.gdiag_host[i] * static_cast<double>(per_class);
    HIPCHK(c, launch_gclass_dot(false, q, L.N, L.gdsqrt, v, c->part, c->part_cap, c->scal + S_TMP, s));
  } else {
    const int64_t per_class = n / (q * q * q);
    for (int i = 0; i < q * q * q; ++i) w0w0 += L.tab.diag[i] * static_cast<double>(per_class);
    HIPCHK(c, launch_class_dot(false, q, L.N, L.tab.dsqrt, v, c->part, c->part_cap, c->scal + S_TMP, s));
  }
  double hs[kNumScal];
  STCHK(read_scalars(c, hs, kNumScal));
  if (L.oct) HIPCHK(c, launch_axpy(false, n, -hs[S_TMP] / w0w0, L.dsqrt64, v, s));
  else if (L.gen) HIPCHK(c, launch_gclass_axpy(q, L.N, L.gdsqrt, -hs[S_TMP] / w0w0, static_cast<double*>(v), s));
  else HIPCHK(c, launch_class_axpy(false, q, L.N, L.tab.dsqrt, -hs[S_TMP] / w0w0, v, s));
  HIPCHK(c, launch_dot(false, n, v, v, c->part, c->scal + S_TMP, s));
  STCHK(read_scalars(c, hs, kNumScal));
  HIPCHK(c, scale(ones, nullptr, nullptr, 1.0 / std::sqrt(hs[S_TMP]), v, v));
  HIPCHK(c, launch_fill_zero(false, n, vprev, s));
  const int steps = static_cast<int>(std::min<int64_t>(c->opt.lanczos_steps, n - 1));
  std::vector<double> alpha, beta;
  double bprev = 0.0, amax = 0.0;
  for (int j = 0; j < steps; ++j) {
    HIPCHK(c, scale(L.tab.dinv_sqrt, L.dinv_sqrt64, L.gdinv_sqrt, 1.0, v, t));
    STCHK(apply_op(c, l, 0, Epi::Apply, t, w, nullptr, nullptr, 0, 0));
    HIPCHK(c, scale(L.tab.dinv_sqrt, L.dinv_sqrt64, L.gdinv_sqrt, 1.0, w, w));
    if (bprev != 0.0) HIPCHK(c, launch_axpy(false, n, -bprev, vprev, w, s));
    HIPCHK(c, launch_dot(false, n, w, v, c->part, c->scal + S_TMP, s));
    STCHK(read_scalars(c, hs, kNumScal));
    const double a = hs[S_TMP];
    alpha.push_back(a);
    amax = std::max(amax, std::fabs(a));
    HIPCHK(c, launch_axpy(false, n, -a, v, w, s));
    HIPCHK(c, launch_dot(false, n, w, w, c->part, c->scal + S_TMP, s));
    STCHK(read_scalars(c, hs, kNumScal));
    const double bnew = std::sqrt(hs[S_TMP]);
    if (j == steps - 1 || bnew <= 1e-12 * amax) break;
    beta.push_back(bnew);
    // vprev <- v ; v <- w / bnew
    std::swap(v, vprev);
    HIPCHK(c, scale(ones, nullptr, nullptr, 1.0 / bnew, w, v));
    bprev = bnew;
  }
  *lam_out = tridiag_max_eig(alpha, beta);
  return GMG_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// zero integral: u <- u - (int u_h) / |cube| on level l (FP64)
gmg_status zero_integral(gmg_ctx* c, int l, void* u) {
  const Level& F = c->lv[l];
  const int64_t n = F.size;
  if (F.oct) HIPCHK(c, launch_dot(false, n, F.wint64, u, c->part, c->scal + S_TMP, c->stream));
  else if (F.gen)
    HIPCHK(c, launch_gclass_dot(false, c->q, F.N, F.gwint, u, c->part, c->part_cap, c->scal + S_TMP, c->stream));
  else HIPCHK(c, launch_class_dot(false, c->q, F.N, F.tab.wint, u, c->part, c->part_cap, c->scal + S_TMP, c->stream));
  HIPCHK(c, launch_shift(false, n, c->scal, S_TMP, 1.0, u, c->stream));
  return GMG_OK;
}

// Preconditioned Krylov solve of A c = r on the finest level in precision pi,
// c = 0 initially.  r is overwritten with the recursive residual.  Stops when
// ||r||_2 <= tol_abs.  With b_true, the stop is confirmed on the true residual
// b_true - A c (and r is reset to it if that is above tolerance).  The
// convergence test comes right after the residual update, so no V-cycle is
// spent on a residual that already meets the tolerance.
//
// norm_slot >= 0: tol_abs is relative to sqrt(scal[norm_slot]) (a norm the caller
// enqueued, read back together with the first residual norm), which goes to *norm.
gmg_status krylov(gmg_ctx* c, int pi, int vpi, bool flexible, const void* b_true, void* u, void* r, double tol_abs,
                  int maxit, int* iters, double* final_rr, int norm_slot = -1, double* norm = nullptr,
                  bool start_from_b = false) {
  const int l = c->L - 1;
  const int64_t n = c->lv[l].size;
  const bool f32 = pi == 1;
  const hipStream_t s = c->stream;
  void* z = c->kz[pi];
  void* p = c->kp[pi];
  void* w = c->kw[pi];
  double hs[kNumScal];
  int rz = S_RZ0;
  // FCG in FP64 around plain FP32 cycles: the residual update, its projection
  // and its cast to FP32 are one pass (the mean it removes is predicted from
  // sum(r) and sum(w), reduced with the step's products; the stored residual's
  // exact sum keeps the norm and the next prediction exact), and the direction
  // updates read the cycle's FP32 output directly (no FP64 copy of z)
  const bool mixed = pi == 0 && vpi == 1 && flexible && r == c->kr[0];
  // the learned cycle in that loop: z32 = V_L r32 under its per-cycle test (and the plain
  // cycle on a fallback) takes the place of the captured plain cycle; the vector work
  // after it is the same
  const bool lrn = mixed && learned_precond(c, vpi);
  bool lrn_pending = false;  // a learned cycle under test is enqueued, not yet decided
  auto lrn_cycle = [&]() -> gmg_status {
    if (!lrn_pending) STCHK(learned_test_enqueue(c, 1, 1, c->kr[1]));
    lrn_pending = false;
    return learned_decide(c, 1, 1, c->kr[1]);
  };
  // on levels the column kernel runs, p.w and sum(w) come out of the apply itself, and
  // p.r is taken as (z - mean z).r: p_old.r = 0 by the choice of alpha, so the two agree
  // in exact arithmetic, and z.r joins the direction update's reduction
  const bool fused_pw = mixed && !c->lv[l].oct && !c->lv[l].gen && c->lv[l].N > 32;
  float* r32 = static_cast<float*>(c->kr[1]);
  const float* z32 = static_cast<const float*>(c->kz[1]);
  *iters = 0;
  const double inv_n = 1.0 / static_cast<double>(n);
  // r <- r - mean(r) and ||r||^2 -> S_RR (mixed: r32 = float(r) in the same pass)
  auto project_norm = [&]() -> gmg_status {
    if (mixed) {
      HIPCHK(c, launch_sum(false, n, r, c->part, c->scal + S_SUM, s));
      HIPCHK(c, launch_shift_cast_sq(n, c->scal, S_SUM, inv_n, static_cast<const double*>(r), static_cast<double*>(r),
                                     r32, c->part, S_RR, S_RS, s));
      return GMG_OK;
    }
    STCHK(project(c, pi, n, r));
    HIPCHK(c, launch_dot(f32, n, r, r, c->part, c->scal + S_RR, s));
    return GMG_OK;
  };
  // first direction p = z - mean(z), z = V r
  // (mixed: the cycle and the vector work after it are one captured sequence; every
  // argument is fixed for the context)
  auto restart = [&]() -> gmg_status {
    if (mixed) {
      if (lrn) STCHK(lrn_cycle());
      return graph_run(c, lrn ? 9 : 7, [&]() -> gmg_status {
        if (!lrn) STCHK(vcycle_seq(c, 1, 1, c->kr[1], c->kz[1]));  // z32 = V r32
        if (fused_pw) {
          HIPCHK(c, launch_sums3_mixed(n, z32, static_cast<const double*>(r), c->part, c->scal, S_ZS, S_ZR, S_YS, s));
          HIPCHK(c, launch_combine(c->scal, S_PR, S_ZR, S_ZS, S_RS, inv_n, s));
        } else {
          HIPCHK(c, launch_sum(true, n, z32, c->part, c->scal + S_ZS, s));
        }
        HIPCHK(c, launch_shift_f2d(n, c->scal, S_ZS, inv_n, z32, static_cast<double*>(p), s));
        return GMG_OK;
      });
    }
    STCHK(precondition(c, pi, vpi, r, z));
    STCHK(project(c, pi, n, z));
    if (!flexible) HIPCHK(c, launch_dot(f32, n, r, z, c->part, c->scal + rz, s));
    HIPCHK(c, launch_copy(f32, n, z, p, s));
    return GMG_OK;
  };
  // the mixed solve's next cycle and direction update (z = V r, p = (z - mean z) + beta p)
  auto mixed_direction = [&]() -> gmg_status {
    if (lrn) STCHK(lrn_cycle());
    return graph_run(c, lrn ? 10 : 8, [&]() -> gmg_status {
      if (!lrn) STCHK(vcycle_seq(c, 1, 1, c->kr[1], c->kz[1]));  // z32 = V r32
      if (fused_pw) {
        HIPCHK(c, launch_sums4_mixed(n, z32, static_cast<const double*>(w), static_cast<const double*>(r), c->part,
                                     c->scal, S_ZS, S_ZW, S_YS, S_ZR, s));
        HIPCHK(c, launch_combine(c->scal, S_PR, S_ZR, S_ZS, S_RS, inv_n, s));
      } else {
        HIPCHK(c, launch_sums3_mixed(n, z32, static_cast<const double*>(w), c->part, c->scal, S_ZS, S_ZW, S_YS, s));
      }
      HIPCHK(c, launch_combine(c->scal, S_ZWC, S_ZW, S_ZS, S_YS, inv_n, s));
      HIPCHK(c, launch_xpby_shift_mixed(n, c->scal, S_ZWC, S_PW, -1.0, S_ZS, inv_n, z32, static_cast<double*>(p), s));
      return GMG_OK;
    });
  };
  // Mixed solves enqueue the cycle that follows a residual update before the host
  // has read the residual's norm, whenever the last norm was more than kSpecMargin
  // times the tolerance (no cycle contracts that much): the host's round trip then
  // overlaps the cycle instead of leaving the device idle.  The speculative work
  // writes only z, p and direction scalars, so on a converged residual it is
  // simply dropped.
  constexpr double kSpecMargin = 1e3;
  bool have_dir = false;
  bool end_pending = false;  // the final check is already enqueued
  if (start_from_b && mixed && norm_slot >= 0) {
    // u = 0 with sum(b) and b.b (the caller's norm) in one pass; r = b - mean(b),
    // its FP32 cast and its sums in the next
    HIPCHK(c, launch_zero_sums(n, static_cast<const double*>(b_true), static_cast<double*>(u), c->part, c->scal,
                               S_SUM, norm_slot, s));
    HIPCHK(c, launch_shift_cast_sq(n, c->scal, S_SUM, inv_n, static_cast<const double*>(b_true),
                                   static_cast<double*>(r), r32, c->part, S_RR, S_RS, s));
  } else {
    if (start_from_b) {
      if (norm_slot >= 0) HIPCHK(c, launch_dot(f32, n, b_true, b_true, c->part, c->scal + norm_slot, s));
      HIPCHK(c, launch_copy(f32, n, b_true, r, s));
    }
    HIPCHK(c, launch_fill_zero(f32, n, u, s));
    STCHK(project_norm());
  }
  const bool speculate = mixed && !c->opt.no_speculation;
  if (speculate) {
    STCHK(scalars_async(c, kNumScal));
    if (lrn) {  // only the cycle under test; its decision waits for the norm
      STCHK(learned_test_enqueue(c, 1, 1, c->kr[1]));
      lrn_pending = true;
    } else {
      STCHK(restart());
      have_dir = true;
    }
    STCHK(scalars_wait(c, hs, kNumScal));
  } else {
    STCHK(read_scalars(c, hs, kNumScal));
  }
  if (norm_slot >= 0) {
    const double nb = std::sqrt(hs[norm_slot]);
    if (norm) *norm = nb;
    if (!std::isfinite(nb)) return fail(c, GMG_E_BREAKDOWN, "load vector is not finite");
    tol_abs *= nb;
    if (nb == 0.0) {  // u = 0 solves it
      *final_rr = 0.0;
      return GMG_OK;
    }
  }
  double rr = hs[S_RR];
  c->hist_res.push_back(std::sqrt(rr));
  int it = 0;
  while (true) {
    if (!std::isfinite(rr)) {
      *iters = it;
      *final_rr = rr;
      return fail(c, GMG_E_BREAKDOWN, "Krylov breakdown: non-finite residual");
    }
    if (std::sqrt(rr) <= tol_abs) {
      lrn_pending = false;  // a speculative learned cycle is dropped with its residual
      if (!b_true) break;
      if (fused_pw) {
        // the true residual (into the unused FP64 z buffer) with its sums from the
        // apply, unless it was enqueued behind the last read-back already; the
        // projection and cast follow only if it is not below the tolerance
        if (!end_pending)
          STCHK(apply_op(c, l, pi, Epi::ResidualSums, u, c->kz[0], b_true, nullptr, 0, 0, false, nullptr, 0.0, S_TR,
                         S_TS));
        end_pending = false;
        STCHK(read_scalars(c, hs, kNumScal));
        rr = std::max(0.0, hs[S_TR] - hs[S_TS] * hs[S_TS] / static_cast<double>(n));
        if (!std::isfinite(hs[S_TR])) rr = hs[S_TR];
        if ((std::sqrt(rr) <= tol_abs && std::isfinite(rr)) || it >= maxit) break;
        HIPCHK(c, launch_copy(false, n, c->kz[0], r, s));
        STCHK(project_norm());
        STCHK(read_scalars(c, hs, kNumScal));
        rr = hs[S_RR];
        have_dir = false;
        continue;
      }
      STCHK(apply_op(c, l, pi, Epi::Residual, u, r, b_true, nullptr, 0, 0));
      STCHK(project_norm());
      STCHK(read_scalars(c, hs, kNumScal));
      rr = hs[S_RR];
      if (std::sqrt(rr) <= tol_abs || it >= maxit) break;
      have_dir = false;
      continue;
    }
    if (it >= maxit) break;
    if (!have_dir) {
      STCHK(restart());
      have_dir = true;
    }
    if (fused_pw) STCHK(apply_op(c, l, pi, Epi::ApplyDot, p, w, nullptr, nullptr, 0, 0, false, nullptr, 0.0, S_PW, S_WS));
    else STCHK(apply_op(c, l, pi, Epi::Apply, p, w, nullptr, nullptr, 0, 0));
    // u += alpha p, r -= alpha w, with sum(r) and r.r of the new r in the same pass;
    // the projection r <- r - mean(r) follows (mixed: is folded in), and
    // ||r - mean||^2 = r.r - (sum r)^2 / n
    int sum_slot = S_SUM;
    if (mixed) {
      if (!fused_pw)
        HIPCHK(c, launch_dot2_sumy(n, static_cast<const double*>(p), static_cast<const double*>(w),
                                   static_cast<const double*>(r), c->part, c->scal, S_PW, S_PR, S_WS, s));
      HIPCHK(c, launch_axpy2_cast(n, c->scal, S_PR, S_PW, S_RS, S_WS, inv_n, static_cast<double*>(u),
                                  static_cast<const double*>(p), static_cast<double*>(r),
                                  static_cast<const double*>(w), r32, c->part, S_RR, s));
      sum_slot = S_RS;
    } else {
      if (flexible) HIPCHK(c, launch_dot2(f32, n, p, w, r, c->part, c->scal, S_PW, S_PR, s));
      else HIPCHK(c, launch_dot(f32, n, p, w, c->part, c->scal + S_PW, s));
      HIPCHK(c, launch_axpy2_sums(f32, n, c->scal, flexible ? S_PR : rz, S_PW, u, p, r, w, c->part, S_SUM, S_RR, s));
      HIPCHK(c, launch_shift(f32, n, c->scal, S_SUM, inv_n, r, s));
    }
    const bool spec = speculate && std::isfinite(rr) && std::sqrt(rr) > kSpecMargin * tol_abs;
    if (spec && lrn) {
      // the learned cycle under test goes behind the read-back; its decision (a second
      // read-back) and the direction update wait for the norm
      STCHK(scalars_async(c, kNumScal));
      STCHK(learned_test_enqueue(c, 1, 1, c->kr[1]));
      lrn_pending = true;
      STCHK(scalars_wait(c, hs, kNumScal));
    } else if (spec) {
      STCHK(scalars_async(c, kNumScal));
      STCHK(mixed_direction());
      STCHK(scalars_wait(c, hs, kNumScal));
    } else if (speculate && fused_pw && b_true) {
      // near the tolerance: the true-residual check goes behind the read-back instead
      // (it writes only the scratch vector and its two sums; if the iteration goes
      // on, they are dropped)
      STCHK(scalars_async(c, kNumScal));
      STCHK(apply_op(c, l, pi, Epi::ResidualSums, u, c->kz[0], b_true, nullptr, 0, 0, false, nullptr, 0.0, S_TR, S_TS));
      end_pending = true;
      STCHK(scalars_wait(c, hs, kNumScal));
    } else {
      STCHK(read_scalars(c, hs, kNumScal));
    }
    rr = std::max(0.0, hs[S_RR] - hs[sum_slot] * hs[sum_slot] / static_cast<double>(n));
    if (!std::isfinite(hs[S_RR])) rr = hs[S_RR];
    c->hist_res.push_back(std::sqrt(rr));
    ++it;
    if (!finite_pos(hs[S_PW])) {
      *iters = it;
      *final_rr = rr;
      return fail(c, GMG_E_BREAKDOWN, "Krylov breakdown: p^T A p <= 0 or not finite");
    }
    if (std::sqrt(rr) <= tol_abs) continue;
    end_pending = false;
    // z is projected inside the direction update: p = (z - mean z) + beta p, with
    // (z - mean z).y = z.y - (sum z)(sum y) / n (y = w for FCG, y = r for PCG)
    if (mixed) {
      if (!spec || lrn) STCHK(mixed_direction());
      continue;
    }
    STCHK(precondition(c, pi, vpi, r, z));
    if (flexible) {
      HIPCHK(c, launch_sums3(f32, n, z, w, c->part, c->scal, S_ZS, S_ZW, S_YS, s));
      HIPCHK(c, launch_combine(c->scal, S_ZWC, S_ZW, S_ZS, S_YS, inv_n, s));
      HIPCHK(c, launch_xpby_shift(f32, n, c->scal, S_ZWC, S_PW, -1.0, S_ZS, inv_n, z, p, s));
    } else {
      const int rzn = rz == S_RZ0 ? S_RZ1 : S_RZ0;
      HIPCHK(c, launch_sums3(f32, n, z, r, c->part, c->scal, S_ZS, rzn, S_YS, s));
      HIPCHK(c, launch_combine(c->scal, rzn, rzn, S_ZS, S_YS, inv_n, s));
      HIPCHK(c, launch_xpby_shift(f32, n, c->scal, rzn, rz, 1.0, S_ZS, inv_n, z, p, s));
      rz = rzn;
    }
  }
  *iters = it;
  *final_rr = rr;
  return GMG_OK;
}

gmg_status check_level(const gmg_ctx* c, int level) {
  if (level < 0 || level >= c->L) return GMG_E_ARG;
  return GMG_OK;
}

}  // namespace

extern "C" {

const char* gmg_status_string(gmg_status s) {
  switch (s) {
    case GMG_OK: return "ok";
    case GMG_E_ARG: return "invalid argument";
    case GMG_E_MESH: return "invalid mesh";
    case GMG_E_OOM: return "out of device memory";
    case GMG_E_HIP: return "HIP runtime error";
    case GMG_E_NOCONV: return "not converged";
    case GMG_E_BREAKDOWN: return "breakdown";
    case GMG_E_STATE: return "invalid state";
  }
  return "unknown status";
}

const char* gmg_last_error(const gmg_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

}  // extern "C"

namespace {

constexpr int kOctCoarsest = 2;  // the octree hierarchy ends at the uniform mesh of this level

// Host side of one octree level.
struct OctHost {
  oct::Space sp;
  std::vector<double> diag, wint;
  oct::Csr P;  // prolongation from the next coarser level (empty on level 0)
};

// Validate the caller's octree and build the hierarchy (finest last):
// coarsening by sibling merge and 2:1 balance (Section 2.3.1) down to the
// uniform mesh of level kOctCoarsest, or `levels` meshes when levels > 0.
gmg_status octree_hierarchy(const gmg_mesh* mesh, int q, std::vector<OctHost>* lv, std::string* err) {
  if (q != 1 && q != 2) {
    *err = "octree meshes support orders 1 and 2";
    return GMG_E_ARG;
  }
  if (mesh->n_leaves <= 0 || !mesh->leaf_morton || !mesh->leaf_level) return GMG_E_ARG;
  std::vector<oct::Leaf> t(static_cast<size_t>(mesh->n_leaves));
  for (int64_t i = 0; i < mesh->n_leaves; ++i) {
    uint32_t x, y, z;
    const uint64_t k = mesh->leaf_morton[i];
    if (k >> (3 * oct::kMaxLevel)) {
      *err = "Morton key beyond the finest level";
      return GMG_E_MESH;
    }
    oct::morton_decode(k, &x, &y, &z);
    t[i] = {static_cast<int32_t>(x), static_cast<int32_t>(y), static_cast<int32_t>(z), mesh->leaf_level[i]};
    if (t[i].level < kOctCoarsest || t[i].level > oct::kMaxLevel) {
      *err = "leaf level outside [2, 10]";
      return GMG_E_MESH;
    }
  }
  if (!oct::is_complete(t)) {
    *err = "octree leaves are not sorted, aligned and complete";
    return GMG_E_MESH;
  }
  if (!oct::is_balanced(t)) {
    *err = "octree is not 2:1 balanced";
    return GMG_E_MESH;
  }
  std::vector<std::vector<oct::Leaf>> trees{t};
  auto uniform_coarsest = [](const std::vector<oct::Leaf>& tr) {
    for (const auto& o : tr)
      if (o.level != kOctCoarsest) return false;
    return true;
  };
  while (!uniform_coarsest(trees.back())) trees.push_back(oct::coarsen(trees.back(), kOctCoarsest));
  std::reverse(trees.begin(), trees.end());
  if (mesh->levels > 0) {
    if (mesh->levels > static_cast<int>(trees.size())) return GMG_E_ARG;
    trees.erase(trees.begin(), trees.end() - mesh->levels);
  }
  std::vector<double> kref, mref;
  oct::reference_element(q, &kref, &mref);
  lv->resize(trees.size());
  for (size_t l = 0; l < trees.size(); ++l) {
    OctHost& h = (*lv)[l];
    h.sp = oct::build_space(trees[l], q);
    h.diag = oct::element_diag_sum(h.sp, kref);
    h.wint = oct::basis_integrals(h.sp, mref);
    if (l > 0) h.P = oct::prolongation((*lv)[l - 1].sp, h.sp);
    if (h.sp.C.col.size() > static_cast<size_t>(INT32_MAX) || h.sp.C.rows > INT32_MAX) return GMG_E_ARG;
  }
  if ((*lv)[0].sp.ndof() > 512) {
    *err = "coarsest octree level has more than 512 DoFs";
    return GMG_E_ARG;
  }
  return GMG_OK;
}

template <typename T>
gmg_status upload(gmg_ctx* c, const std::vector<T>& v, const T** dst) {
  void* p = nullptr;
  STCHK(dalloc(c, &p, sizeof(T) * std::max<size_t>(v.size(), 1)));
  if (!v.empty()) HIPCHK(c, hipMemcpy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  *dst = static_cast<const T*>(p);
  return GMG_OK;
}

std::vector<int> narrow(const std::vector<int64_t>& v) { return std::vector<int>(v.begin(), v.end()); }
std::vector<float> to_f32(const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); }

gmg_status upload_csr(gmg_ctx* c, const oct::Csr& a, const int** ptr, const int** col, const double** v64,
                      const float** v32) {
  STCHK(upload(c, narrow(a.ptr), ptr));
  STCHK(upload(c, a.col, col));
  STCHK(upload(c, a.val, v64));
  STCHK(upload(c, to_f32(a.val), v32));
  return GMG_OK;
}

// Device arrays of octree level l from its host side.
gmg_status upload_octree_level(gmg_ctx* c, Level& L, OctHost& h, const std::vector<double>& kref,
                               const std::vector<double>& mref) {
  L.oct = true;
  L.n = L.N = 0;
  L.size = h.sp.ndof();
  L.leaves = h.sp.leaves;
  L.points = h.sp.points;
  OctLevelDev& d = L.od;
  d.E = h.sp.elements();
  d.n = L.size;
  d.m = h.sp.m;
  std::vector<uint8_t> lev(d.E);
  for (int64_t e = 0; e < d.E; ++e) lev[e] = static_cast<uint8_t>(h.sp.leaves[e].level);
  STCHK(upload(c, lev, &d.lev));
  STCHK(upload_csr(c, h.sp.C, &d.cptr, &d.ccol, &d.cval64, &d.cval32));
  STCHK(upload_csr(c, oct::transpose(h.sp.C), &d.tptr, &d.trow, &d.tval64, &d.tval32));
  STCHK(upload(c, kref, &d.kref64));
  STCHK(upload(c, to_f32(kref), &d.kref32));
  STCHK(upload(c, mref, &d.mref64));
  STCHK(upload(c, to_f32(mref), &d.mref32));
  std::vector<double> dinv(L.size), dsq(L.size), dis(L.size);
  L.w0w0 = 0.0;
  for (int64_t k = 0; k < L.size; ++k) {
    if (!(h.diag[k] > 0.0)) return fail(c, GMG_E_MESH, "non-positive diagonal entry on an octree level");
    dinv[k] = 1.0 / h.diag[k];
    dsq[k] = std::sqrt(h.diag[k]);
    dis[k] = 1.0 / dsq[k];
    L.w0w0 += h.diag[k];
  }
  STCHK(upload(c, dinv, &d.dinv64));
  STCHK(upload(c, to_f32(dinv), &d.dinv32));
  const double* p = nullptr;
  STCHK(upload(c, h.diag, &p));
  L.diag64 = const_cast<double*>(p);
  STCHK(upload(c, dsq, &p));
  L.dsqrt64 = const_cast<double*>(p);
  STCHK(upload(c, dis, &p));
  L.dinv_sqrt64 = const_cast<double*>(p);
  STCHK(upload(c, h.wint, &p));
  L.wint64 = const_cast<double*>(p);
  // leaves all of one level: the DoFs are the uniform lattice of 2^level elements a side
  bool one_level = !h.sp.leaves.empty();
  for (const auto& lf : h.sp.leaves) one_level = one_level && lf.level == h.sp.leaves[0].level;
  if (one_level) {
    const int ne = 1 << h.sp.leaves[0].level;
    if (static_cast<int64_t>(c->q * ne) * (c->q * ne) * (c->q * ne) == L.size) {
      L.latN = c->q * ne;
      L.tab = make_level_tables(c->q, ne);
    }
  }
  if (h.P.rows > 0) {
    STCHK(upload_csr(c, h.P, &d.pptr, &d.pcol, &d.pval64, &d.pval32));
    STCHK(upload_csr(c, oct::transpose(h.P), &d.rptr, &d.rcol, &d.rval64, &d.rval32));
  }
  c->oye_size = std::max<int64_t>(c->oye_size, d.E * d.m);
  return GMG_OK;
}

// Device tables of a uniform level of an order without a specialised kernel.
gmg_status upload_generic_level(gmg_ctx* c, Level& L) {
  const GenTables T = make_generic_tables(c->q, L.n);
  L.gen = true;
  L.latN = 0;  // the learned smoother runs on q <= 4 lattices only
  for (GenOp* op : {&L.gstiff, &L.gmass}) {
    const std::vector<double>& rows = op == &L.gstiff ? T.stiff_rows : T.mass_rows;
    op->q = c->q;
    STCHK(upload(c, rows, &op->rows64));
    STCHK(upload(c, to_f32(rows), &op->rows32));
    STCHK(upload(c, T.dinv, &op->dinv64));
    STCHK(upload(c, to_f32(T.dinv), &op->dinv32));
  }
  STCHK(upload(c, T.diag, &L.gdiag));
  STCHK(upload(c, T.dsqrt, &L.gdsqrt));
  STCHK(upload(c, T.dinv_sqrt, &L.gdinv_sqrt));
  STCHK(upload(c, T.wint, &L.gwint));
  L.gdiag_host = T.diag;
  return GMG_OK;
}

}  // namespace

extern "C" {

gmg_status gmg_setup(const gmg_mesh* mesh, const gmg_options* opts, void* hip_stream, gmg_ctx** out) {
  if (!mesh || !out) return GMG_E_ARG;
  *out = nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  const int q = mesh->order;
  const int n = mesh->n;
  const bool octree = n == 0;
  // q = 1, 2, 4 run the specialised kernels; 3 and 5 .. 16 the generic ones (uniform meshes)
  const bool gen = q == 3 || (q >= 5 && q <= kGenMaxQ);
  if (!(q == 1 || q == 2 || q == 4 || gen)) return GMG_E_ARG;
  if (gen && n == 0) return GMG_E_ARG;  // octree meshes: orders 1 and 2
  int L = mesh->levels;
  int nc0 = 0;
  int64_t n0 = 0;
  std::vector<OctHost> oh;
  std::string oerr;
  if (octree) {
    gmg_status st;
    try {
      st = octree_hierarchy(mesh, q, &oh, &oerr);
    } catch (const std::bad_alloc&) {
      return GMG_E_OOM;
    } catch (...) {
      return GMG_E_MESH;
    }
    if (st != GMG_OK) return st;
    L = static_cast<int>(oh.size());
    n0 = oh[0].sp.ndof();
  } else {
    // the generic orders go down to a single periodic element (where coarsening ends,
    // Section 2.3.1); q = 1, 2, 4 keep at least two elements a side
    const int nmin = gen ? 1 : 2;
    const int Nmin = gen ? 3 : 4;  // lattice nodes a side: the shapes of the q = 1, 2, 4 kernels need 4
    if (n < nmin || (n & (n - 1)) != 0 || q * n < Nmin || n > (gen ? 64 : (q == 4 ? 256 : 512))) return GMG_E_ARG;
    if (L <= 0) {
      L = 1;
      // deepest hierarchy with coarsest level >= nmin elements and <= 512 DoFs
      while (true) {
        const int nc = n >> (L - 1);
        const int64_t dofs = static_cast<int64_t>(q * nc) * (q * nc) * (q * nc);
        if (dofs <= 512 || nc / 2 < nmin || q * (nc / 2) < Nmin) break;
        ++L;
      }
    }
    if ((n >> (L - 1)) < 1 || (n >> (L - 1)) << (L - 1) != n) return GMG_E_ARG;
    nc0 = n >> (L - 1);
    if (q * nc0 < Nmin || nc0 < nmin) return GMG_E_ARG;
    n0 = static_cast<int64_t>(q * nc0) * (q * nc0) * (q * nc0);
    // dense FP64 coarsest solve: at most 512 DoFs, or one periodic element of order up to
    // 16 (at most 4096 DoFs, its pseudo-inverse formed from the 1D eigenpairs)
    if (n0 > (nc0 == 1 ? 4096 : 512)) return GMG_E_ARG;
  }

  gmg_ctx* c = new (std::nothrow) gmg_ctx();
  if (!c) return GMG_E_OOM;
  c->q = q;
  c->L = L;
  c->octree = octree;
  c->gen = gen;
  gmg_options o{};
  if (opts) o = *opts;
  if (o.cheb_degree <= 0) o.cheb_degree = 3;
  if (o.nu_pre <= 0 && !(opts && opts->nu_pre < 0)) o.nu_pre = 2;
  if (o.nu_post <= 0 && !(opts && opts->nu_post < 0)) o.nu_post = 2;
  if (o.nu_pre < 0) o.nu_pre = 0;
  if (o.nu_post < 0) o.nu_post = 0;
  if (o.cheb_lo <= 0) o.cheb_lo = 0.1;
  if (o.cheb_hi <= 0) o.cheb_hi = 1.1;
  if (o.lanczos_steps <= 0) o.lanczos_steps = 10;
  if (o.jacobi_omega <= 0) o.jacobi_omega = 2.0 / 3.0;
  if (o.inner_rtol <= 0) o.inner_rtol = 2e-6;
  if (o.max_iters <= 0) o.max_iters = 500;
  if (o.use_learned) o.vcycle_prec = GMG_FP32;  // the learned cycle is an FP32 cycle
  if (o.vcycle_prec == GMG_FP32) o.krylov = 1;
  c->opt = o;
  c->user = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&c->device) != hipSuccess) {
    gmg_destroy(c);
    return GMG_E_HIP;
  }
  // the device address of gmg_dot_noalloc's static scratch, once per device
  if (noalloc_scratch_init(c->device) != hipSuccess) {
    gmg_destroy(c);
    return GMG_E_HIP;
  }
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    c->stream = nullptr;
    gmg_destroy(c);
    return GMG_E_HIP;
  }
  if (hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_copy, hipEventDisableTiming) != hipSuccess ||
      hipEventCreate(&c->ev_t0) != hipSuccess || hipEventCreate(&c->ev_t1) != hipSuccess) {
    gmg_destroy(c);
    return GMG_E_HIP;
  }
  if (hipEventRecord(c->ev_in, c->user) != hipSuccess || hipStreamWaitEvent(c->stream, c->ev_in, 0) != hipSuccess) {
    gmg_destroy(c);
    return GMG_E_HIP;
  }
  c->lv.resize(L);
  c->nets.resize(L);
  c->net_set.assign(L, 0);
  c->lcache.assign(L, nullptr);
  c->tsec.assign(static_cast<size_t>(L) * kKinds * 2, 0.0);
  c->tcount.assign(static_cast<size_t>(L) * kKinds * 2, 0);
  gmg_status st = GMG_OK;
  auto bail = [&](gmg_status s) {
    gmg_destroy(c);
    return s;
  };
  if (octree) {
    std::vector<double> kref, mref;
    oct::reference_element(q, &kref, &mref);
    for (int l = 0; l < L; ++l)
      if ((st = upload_octree_level(c, c->lv[l], oh[l], kref, mref)) != GMG_OK) return bail(st);
    // apply scratch of both precisions (every entry point that applies an operator needs it)
    for (int pi = 0; pi < 2; ++pi)
      if ((st = dalloc(c, &c->oye[pi], c->oye_size * esize(pi))) != GMG_OK) return bail(st);
  } else {
    for (int l = 0; l < L; ++l) {
      Level& lev = c->lv[l];
      lev.n = n >> (L - 1 - l);
      lev.N = q * lev.n;
      lev.size = static_cast<int64_t>(lev.N) * lev.N * lev.N;
      if (gen) {
        if ((st = upload_generic_level(c, lev)) != GMG_OK) return bail(st);
        continue;
      }
      lev.latN = lev.N;
      lev.tab = make_level_tables(q, lev.n);
      prime_apply_shapes(q, lev.N);
      if (l + 1 < L) prime_transfer_shapes(q, lev.N);  // restriction onto this level
    }
    if (gen) {
      std::vector<double> p, r;
      make_generic_transfer(q, &p, &r);
      c->gxfer.q = q;
      if ((st = upload(c, p, &c->gxfer.p)) != GMG_OK || (st = upload(c, r, &c->gxfer.r)) != GMG_OK) return bail(st);
    } else {
      make_transfer_table(q, &c->xfer);
    }
  }
  if ((st = dalloc(c, reinterpret_cast<void**>(&c->scal), sizeof(double) * kNumScal)) != GMG_OK) return bail(st);
  if (hipHostMalloc(reinterpret_cast<void**>(&c->scal_host), sizeof(double) * kNumScal, hipHostMallocDefault) !=
      hipSuccess) {
    c->scal_host = nullptr;
    return bail(fail(c, GMG_E_OOM, "hipHostMalloc of the scalar read-back buffer failed"));
  }
  {
    // N^2 row partials of the finest level, plus room for their first folding pass
    const int64_t rows = static_cast<int64_t>(c->lv.back().N) * c->lv.back().N;
    c->part_cap = std::max<int64_t>(3 * kRedBlocks, rows + rows / 64 + 64);
  }
  if ((st = dalloc(c, reinterpret_cast<void**>(&c->part), sizeof(double) * c->part_cap)) != GMG_OK) return bail(st);
  if (hipMemsetAsync(c->scal, 0, sizeof(double) * kNumScal, c->stream) != hipSuccess) return bail(GMG_E_HIP);
  if ((st = ensure_prec(c, 0)) != GMG_OK) return bail(st);
  // coarsest pseudo-inverse
  c->n0 = static_cast<int>(n0);
  std::vector<double> inv;
  try {
    if (octree) {
      std::vector<double> kref, mref;
      oct::reference_element(q, &kref, &mref);
      inv = dense_pseudo_inverse(oct::dense_operator(oh[0].sp, kref), static_cast<int>(n0));
      oh.clear();
    } else {
      inv = coarse_pseudo_inverse(q, nc0);
    }
  } catch (...) {
    return bail(GMG_E_ARG);
  }
  if ((st = dalloc(c, reinterpret_cast<void**>(&c->ainv), sizeof(double) * inv.size())) != GMG_OK) return bail(st);
  if (hipMemcpyAsync(c->ainv, inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice, c->stream) !=
          hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return bail(GMG_E_HIP);
  // Chebyshev interval per level
  for (int l = 0; l < L; ++l) {
    Level& lev = c->lv[l];
    double lam = o.lambda_override;
    if (lam <= 0.0) {
      if ((st = lanczos(c, l, &lam)) != GMG_OK) return bail(st);
    }
    lev.lam = lam;
    lev.alpha = o.cheb_lo * lam;
    lev.beta = o.cheb_hi * lam;
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(GMG_E_HIP);
  c->t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = c;
  return GMG_OK;
}

gmg_status gmg_destroy(gmg_ctx* ctx) {
  if (!ctx) return GMG_OK;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  for (hipGraphExec_t g : ctx->vgraph)
    if (g) (void)hipGraphExecDestroy(g);
  for (void* p : ctx->allocs) (void)hipFree(p);
  if (ctx->scal_host) (void)hipHostFree(ctx->scal_host);
  for (hipEvent_t e : ctx->ev_all) (void)hipEventDestroy(e);
  if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
  if (ctx->ev_t0) (void)hipEventDestroy(ctx->ev_t0);
  if (ctx->ev_t1) (void)hipEventDestroy(ctx->ev_t1);
  if (ctx->ev_out) (void)hipEventDestroy(ctx->ev_out);
  if (ctx->ev_copy) (void)hipEventDestroy(ctx->ev_copy);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return GMG_OK;
}

gmg_status gmg_num_levels(const gmg_ctx* ctx, int32_t* levels) {
  if (!ctx || !levels) return GMG_E_ARG;
  *levels = ctx->L;
  return GMG_OK;
}

gmg_status gmg_num_dofs(const gmg_ctx* ctx, int32_t level, int64_t* n) {
  if (!ctx || !n || check_level(ctx, level) != GMG_OK) return GMG_E_ARG;
  *n = ctx->lv[level].size;
  return GMG_OK;
}

gmg_status gmg_dof_coords_1d(const gmg_ctx* ctx, int32_t level, double* x_host) {
  if (!ctx || !x_host || check_level(ctx, level) != GMG_OK || ctx->lv[level].oct) return GMG_E_ARG;
  const Level& L = ctx->lv[level];
  const std::vector<double> xi = lgl_nodes01(ctx->q);
  for (int i = 0; i < L.N; ++i) x_host[i] = (i / ctx->q + xi[i % ctx->q]) / L.n;
  return GMG_OK;
}

gmg_status gmg_lambda(const gmg_ctx* ctx, int32_t level, double* lambda_host) {
  if (!ctx || !lambda_host || check_level(ctx, level) != GMG_OK) return GMG_E_ARG;
  *lambda_host = ctx->lv[level].lam;
  return GMG_OK;
}

gmg_status gmg_diagonal(gmg_ctx* ctx, int32_t level, double* d_dev) {
  if (!ctx || !d_dev || check_level(ctx, level) != GMG_OK) return GMG_E_ARG;
  const Level& L = ctx->lv[level];
  return scoped(ctx, [&] {
    if (L.oct) HIPCHK(ctx, launch_copy(false, L.size, L.diag64, d_dev, ctx->stream));
    else if (L.gen) HIPCHK(ctx, launch_gclass_scale(false, ctx->q, L.N, L.gdiag, 1.0, nullptr, d_dev, ctx->stream));
    else HIPCHK(ctx, launch_class_scale(false, ctx->q, L.N, L.tab.diag, 1.0, nullptr, d_dev, ctx->stream));
    return GMG_OK;
  });
}

gmg_status gmg_apply(gmg_ctx* ctx, int32_t level, gmg_prec prec, const void* x_dev, void* y_dev) {
  if (!ctx || !x_dev || !y_dev || check_level(ctx, level) != GMG_OK) return GMG_E_ARG;
  if (x_dev == y_dev) return fail(ctx, GMG_E_ARG, "apply: x and y must not alias");
  if (ctx->gen) STCHK(ensure_prec(ctx, pidx(prec)));  // the generic passes' temporaries
  return scoped(ctx, [&] { return apply_op(ctx, level, pidx(prec), Epi::Apply, x_dev, y_dev, nullptr, nullptr, 0, 0); });
}

gmg_status gmg_fft_solve(gmg_ctx* ctx, const double* b_dev, double* u_dev) {
  if (!ctx || !b_dev || !u_dev) return GMG_E_ARG;
  if (static_cast<const void*>(b_dev) == static_cast<const void*>(u_dev))
    return fail(ctx, GMG_E_ARG, "FFT solve: b and u must not alias");
  const Level& F = ctx->lv.back();
  if (F.oct) return fail(ctx, GMG_E_ARG, "FFT solve: uniform meshes only");
  if (F.gen) return fail(ctx, GMG_E_ARG, "FFT solve: orders 1, 2 and 4 only");
  if (ctx->q == 1) {
    if (!ctx->fft) ctx->fft.reset(new FftQ1());
    return scoped(ctx, [&]() -> gmg_status {
      HIPCHK(ctx, fft_q1_prepare(ctx->fft.get(), F.N));
      HIPCHK(ctx, fft_q1_solve(ctx->fft.get(), b_dev, u_dev, ctx->stream));
      return GMG_OK;
    });
  }
  if (ctx->q == 2) {
    if (!ctx->fft2) ctx->fft2.reset(new FftQ2());
    return scoped(ctx, [&]() -> gmg_status {
      HIPCHK(ctx, fft_q2_prepare(ctx->fft2.get(), F.n));
      HIPCHK(ctx, fft_q2_solve(ctx->fft2.get(), b_dev, u_dev, ctx->stream));
      return GMG_OK;
    });
  }
  if (!ctx->fft4) ctx->fft4.reset(new FftQ4());
  return scoped(ctx, [&]() -> gmg_status {
    HIPCHK(ctx, fft_q4_prepare(ctx->fft4.get(), F.n));
    HIPCHK(ctx, fft_q4_solve(ctx->fft4.get(), b_dev, u_dev, ctx->stream));
    return GMG_OK;
  });
}

gmg_status gmg_mass(gmg_ctx* ctx, int32_t level, gmg_prec prec, const void* x_dev, void* y_dev) {
  if (!ctx || !x_dev || !y_dev || check_level(ctx, level) != GMG_OK) return GMG_E_ARG;
  if (x_dev == y_dev) return fail(ctx, GMG_E_ARG, "mass: x and y must not alias");
  if (ctx->gen) STCHK(ensure_prec(ctx, pidx(prec)));  // the generic passes' temporaries
  return scoped(ctx, [&] { return apply_op(ctx, level, pidx(prec), Epi::Apply, x_dev, y_dev, nullptr, nullptr, 0, 0, true); });
}

gmg_status gmg_smooth(gmg_ctx* ctx, int32_t level, gmg_prec prec, const void* b_dev, void* u_dev, int32_t nu) {
  if (!ctx || !b_dev || !u_dev || nu < 0 || check_level(ctx, level) != GMG_OK) return GMG_E_ARG;
  const int pi = pidx(prec);
  STCHK(ensure_prec(ctx, pi));
  return scoped(ctx, [&] { return smooth(ctx, level, pi, b_dev, u_dev, nu, false); });
}

gmg_status gmg_restrict(gmg_ctx* ctx, int32_t level, gmg_prec prec, const void* rf_dev, void* rc_dev) {
  if (!ctx || !rf_dev || !rc_dev || level < 1 || check_level(ctx, level) != GMG_OK) return GMG_E_ARG;
  const int pi = pidx(prec);
  STCHK(ensure_prec(ctx, pi));
  return scoped(ctx, [&] { return restrict_level(ctx, level, pi, rf_dev, rc_dev); });
}

gmg_status gmg_prolong(gmg_ctx* ctx, int32_t level, gmg_prec prec, const void* ec_dev, void* uf_dev) {
  if (!ctx || !ec_dev || !uf_dev || level < 1 || check_level(ctx, level) != GMG_OK) return GMG_E_ARG;
  const int pi = pidx(prec);
  STCHK(ensure_prec(ctx, pi));
  return scoped(ctx, [&] { return prolong_level(ctx, level, pi, ec_dev, uf_dev); });
}

gmg_status gmg_coarse_solve(gmg_ctx* ctx, gmg_prec prec, const void* b_dev, void* x_dev) {
  if (!ctx || !b_dev || !x_dev || b_dev == x_dev) return GMG_E_ARG;
  return scoped(ctx, [&] { return coarse_solve(ctx, pidx(prec), b_dev, x_dev); });
}

gmg_status gmg_vcycle(gmg_ctx* ctx, gmg_prec prec, const void* r_dev, void* z_dev) {
  if (!ctx || !r_dev || !z_dev || r_dev == z_dev) return GMG_E_ARG;
  const int pi = pidx(prec);
  STCHK(ensure_prec(ctx, pi));
  return scoped(ctx, [&] { return vcycle_level(ctx, ctx->L - 1, pi, r_dev, z_dev); });
}

gmg_status gmg_rhs(gmg_ctx* ctx, const double* f_dev, double* b_dev) {
  if (!ctx || !f_dev || !b_dev || static_cast<const void*>(f_dev) == static_cast<void*>(b_dev)) return GMG_E_ARG;
  const int l = ctx->L - 1;
  return scoped(ctx, [&] {
    STCHK(apply_op(ctx, l, 0, Epi::Apply, f_dev, b_dev, nullptr, nullptr, 0, 0, true));
    return project(ctx, 0, ctx->lv[l].size, b_dev);
  });
}

gmg_status gmg_dot(gmg_ctx* ctx, gmg_prec prec, int64_t n, const void* x_dev, const void* y_dev, double* out_host) {
  if (!ctx || !x_dev || !y_dev || !out_host || n < 0) return GMG_E_ARG;
  return scoped(ctx, [&] {
    HIPCHK(ctx, launch_dot(prec == GMG_FP32, n, x_dev, y_dev, ctx->part, ctx->scal + S_TMP, ctx->stream));
    double hs[kNumScal];
    STCHK(read_scalars(ctx, hs, kNumScal));
    *out_host = hs[S_TMP];
    return GMG_OK;
  });
}

}  // extern "C"

struct gmg_spectral {
  FftSpectral f;
  hipStream_t stream = nullptr;
};

extern "C" {

gmg_status gmg_spectral_create(int32_t N, void* hip_stream, gmg_spectral** out) {
  if (!out) return GMG_E_ARG;
  *out = nullptr;
  if (!spectral_size_ok(N)) return GMG_E_ARG;
  gmg_spectral* s = new (std::nothrow) gmg_spectral();
  if (!s) return GMG_E_OOM;
  s->stream = static_cast<hipStream_t>(hip_stream);
  const hipError_t e = spectral_prepare(&s->f, N);
  if (e != hipSuccess) {
    delete s;
    return e == hipErrorOutOfMemory ? GMG_E_OOM : GMG_E_HIP;
  }
  *out = s;
  return GMG_OK;
}

gmg_status gmg_spectral_solve(gmg_spectral* sp, const double* f_dev, double* u_dev) {
  if (!sp || !f_dev || !u_dev) return GMG_E_ARG;
  return spectral_solve(sp->f, f_dev, u_dev, sp->stream) == hipSuccess ? GMG_OK : GMG_E_HIP;
}

gmg_status gmg_spectral_destroy(gmg_spectral* sp) {
  delete sp;
  return GMG_OK;
}

gmg_status gmg_dot_noalloc(gmg_ctx* ctx, gmg_prec prec, int64_t n, const void* x_dev, const void* y_dev,
                           double* out_dev) {
  // n = 0 reads nothing (x_dev, y_dev may then be null) and writes 0
  if (!ctx || !out_dev || n < 0 || (n > 0 && (!x_dev || !y_dev))) return GMG_E_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != ctx->device)
    return fail(ctx, GMG_E_ARG, "gmg_dot_noalloc: call with the context's device current");
  return scoped(ctx, [&] {
    const hipError_t e = launch_dot_noalloc(ctx->device, prec == GMG_FP32, n, x_dev, y_dev, out_dev, ctx->stream);
    if (e == hipErrorNotInitialized) return fail(ctx, GMG_E_STATE, "gmg_dot_noalloc: scratch not set up on this device");
    if (e == hipErrorInvalidValue) return fail(ctx, GMG_E_ARG, "gmg_dot_noalloc: more partials than the scratch holds");
    HIPCHK(ctx, e);
    return GMG_OK;
  });
}

}  // extern "C"

namespace {

gmg_status solve_rhs_impl(gmg_ctx* ctx, const double* b_dev, double* u_dev, double rtol, gmg_info* info) {
  gmg_ctx* c = ctx;
  const int l = c->L - 1;
  const int64_t n = c->lv[l].size;
  const hipStream_t s = c->stream;
  gmg_info inf{};
  inf.t_setup = c->t_setup;
  STCHK(prepare_learned(c));
  c->fallbacks = 0;
  c->hist_res.clear();
  c->hist_cyc.clear();
  double ph0[4] = {0.0, 0.0, 0.0, 0.0};
  if (c->opt.timing) {
    STCHK(drain_timing(c));
    phase_totals(c, ph0);
  }
  hipEvent_t e0 = c->ev_t0, e1 = c->ev_t1;
  HIPCHK(c, hipEventRecord(e0, s));
  double hs[kNumScal];
  // the Krylov paths read ||b|| back together with their first residual norm; the
  // FP64 flexible CG around FP32 cycles also computes it in its first pass
  const bool krylov_path = c->opt.vcycle_prec != GMG_FP32 || c->opt.ir_mode == 0;
  const bool mixed_fcg = c->opt.vcycle_prec == GMG_FP32 && c->opt.ir_mode == 0;
  if (!mixed_fcg) HIPCHK(c, launch_dot(false, n, b_dev, b_dev, c->part, c->scal + S_TMP, s));
  double nb = 1.0;
  if (!krylov_path) {
    STCHK(read_scalars(c, hs, kNumScal));
    nb = std::sqrt(hs[S_TMP]);
  }
  gmg_status st = GMG_OK;
  if (!std::isfinite(nb)) {
    st = fail(c, GMG_E_BREAKDOWN, "load vector is not finite");
  } else if (nb == 0.0) {
    HIPCHK(c, launch_fill_zero(false, n, u_dev, s));
  } else if (c->opt.vcycle_prec == GMG_FP32 && c->opt.ir_mode == 0) {
    // FP64 FCG(1) preconditioned by one FP32 V-cycle: the residual update, dots
    // and projection stay in FP64 at every iteration (refinement at each step),
    // the V-cycle -- smoother, transfers, level operators -- runs in FP32.
    STCHK(ensure_prec(c, 1));
    int it = 0;
    double rr = 0.0;
    st = krylov(c, 0, 1, true, b_dev, u_dev, c->kr[0], rtol, c->opt.max_iters, &it, &rr, S_TMP, &nb, true);
    inf.inner_iters = it;
    inf.outer_iters = it;
    inf.rel_residual_f64 = nb > 0.0 ? std::sqrt(rr) / nb : 0.0;
    if (st == GMG_OK && !(inf.rel_residual_f64 <= rtol)) st = fail(c, GMG_E_NOCONV, "max_iters reached");
  } else if (c->opt.vcycle_prec != GMG_FP32) {
    // plain FP64: CG / FCG(1) preconditioned by one FP64 V-cycle
    HIPCHK(c, launch_copy(false, n, b_dev, c->kr[0], s));
    int it = 0;
    double rr = 0.0;
    st = krylov(c, 0, 0, c->opt.krylov == 1, b_dev, u_dev, c->kr[0], rtol, c->opt.max_iters, &it, &rr, S_TMP,
                &nb);
    inf.inner_iters = it;
    inf.rel_residual_f64 = nb > 0.0 ? std::sqrt(rr) / nb : 0.0;
    if (st == GMG_OK && !(inf.rel_residual_f64 <= rtol)) st = fail(c, GMG_E_NOCONV, "max_iters reached");
  } else {
    // FP64 iterative refinement around FP32 FCG(1) with FP32 V-cycles.  Each
    // inner solve reduces its residual by tau = max(inner_rtol, rtol ||b|| / (2 ||r||)):
    // no further than the outer tolerance needs, and not below what FP32
    // arithmetic resolves.
    STCHK(ensure_prec(c, 1));
    HIPCHK(c, launch_fill_zero(false, n, u_dev, s));
    HIPCHK(c, launch_copy(false, n, b_dev, c->kr[0], s));   // r = b - A 0
    int total = 0;
    bool first = true;
    while (true) {
      if (!first) {
        STCHK(apply_op(c, l, 0, Epi::Residual, u_dev, c->kr[0], b_dev, nullptr, 0, 0));
        STCHK(project(c, 0, n, c->kr[0]));
      }
      first = false;
      HIPCHK(c, launch_dot(false, n, c->kr[0], c->kr[0], c->part, c->scal + S_TMP, s));
      STCHK(read_scalars(c, hs, kNumScal));
      const double rn = std::sqrt(hs[S_TMP]);
      inf.rel_residual_f64 = rn / nb;
      if (!std::isfinite(rn)) {
        st = fail(c, GMG_E_BREAKDOWN, "non-finite residual in refinement");
        break;
      }
      if (rn <= rtol * nb) break;
      if (total >= c->opt.max_iters) {
        st = fail(c, GMG_E_NOCONV, "max_iters reached");
        break;
      }
      HIPCHK(c, launch_cast_d2f(n, static_cast<const double*>(c->kr[0]), static_cast<float*>(c->kr[1]), s));
      int it = 0;
      double rr = 0.0;
      const double tau = std::max(c->opt.inner_rtol, 0.5 * rtol * nb / rn);
      const int cap = std::min(c->opt.max_iters - total, 40);
      st = krylov(c, 1, 1, true, nullptr, c->kc[1], c->kr[1], tau * rn, cap, &it, &rr);
      total += it;
      if (st != GMG_OK) break;
      HIPCHK(c, launch_add_f2d(n, static_cast<const float*>(c->kc[1]), u_dev, s));
      ++inf.outer_iters;
      if (it == 0) {
        st = fail(c, GMG_E_NOCONV, "FP32 inner solve made no progress");
        break;
      }
    }
    inf.inner_iters = total;
  }
  if (st == GMG_OK || st == GMG_E_NOCONV) STCHK(zero_integral(c, l, u_dev));
  HIPCHK(c, hipEventRecord(e1, s));
  HIPCHK(c, hipEventSynchronize(e1));
  float ms = 0.0f;
  HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
  inf.t_solve = ms * 1e-3;
  inf.fallbacks = static_cast<int32_t>(c->fallbacks);
  if (c->opt.timing) {
    STCHK(drain_timing(c));
    double ph1[4];
    phase_totals(c, ph1);
    inf.t_smooth = ph1[0] - ph0[0];
    inf.t_transfer = ph1[1] - ph0[1];
    inf.t_coarse = ph1[2] - ph0[2];
    inf.t_learned = ph1[3] - ph0[3];
  }
  if (info) *info = inf;
  return st;
}

}  // namespace

extern "C" {

gmg_status gmg_solve_rhs(gmg_ctx* ctx, const double* b_dev, double* u_dev, double rtol, gmg_info* info) {
  if (!ctx || !b_dev || !u_dev || !(rtol > 0.0)) return GMG_E_ARG;
  return scoped(ctx, [&] { return solve_rhs_impl(ctx, b_dev, u_dev, rtol, info); });
}

gmg_status gmg_timing_get(gmg_ctx* ctx, int32_t level, int32_t kind, gmg_prec prec, int64_t* launches,
                          double* seconds) {
  if (!ctx || !launches || !seconds || check_level(ctx, level) != GMG_OK || kind < 0 || kind >= kKinds)
    return GMG_E_ARG;
  STCHK(drain_timing(ctx));
  const int s = tslot(level, kind, pidx(prec));
  *launches = ctx->tcount[s];
  *seconds = ctx->tsec[s];
  return GMG_OK;
}

namespace {
gmg_status write_leaves(const std::vector<oct::Leaf>& t, uint64_t* morton_out, uint8_t* level_out, int64_t cap,
                        int64_t* n_out) {
  *n_out = static_cast<int64_t>(t.size());
  if (*n_out > cap || !morton_out || !level_out) return GMG_E_ARG;
  for (size_t i = 0; i < t.size(); ++i) {
    morton_out[i] = oct::morton_key(t[i].x, t[i].y, t[i].z);
    level_out[i] = static_cast<uint8_t>(t[i].level);
  }
  return GMG_OK;
}
}  // namespace

gmg_status gmg_octree_refine_gaussians(int32_t base_level, int32_t max_level, int32_t count, const double* centres,
                                       const double* sigma, const double* amps, double tol, uint64_t* morton_out,
                                       uint8_t* level_out, int64_t cap, int64_t* n_out) {
  if (!n_out || count < 0 || (count > 0 && (!centres || !sigma || !amps)) || base_level < 0 ||
      max_level > oct::kMaxLevel || base_level > max_level || !(tol > 0.0))
    return GMG_E_ARG;
  for (int i = 0; i < count; ++i)
    if (!(sigma[i] > 0.0)) return GMG_E_ARG;
  try {
    return write_leaves(oct::refine_gaussians(base_level, max_level, count, centres, sigma, amps, tol), morton_out,
                        level_out, cap, n_out);
  } catch (...) {
    return GMG_E_OOM;
  }
}

gmg_status gmg_octree_refine_sharp_layer(int32_t base_level, int32_t max_level, const double* centre, double radius,
                                         double alpha, double tol, uint64_t* morton_out, uint8_t* level_out,
                                         int64_t cap, int64_t* n_out) {
  if (!n_out || !centre || base_level < 0 || max_level > oct::kMaxLevel || base_level > max_level ||
      !(tol > 0.0) || !(radius > 0.0) || !(alpha > 2.0) || !(alpha <= 1e4))
    return GMG_E_ARG;
  for (int k = 0; k < 3; ++k)
    if (!(centre[k] >= 0.0 && centre[k] < 1.0)) return GMG_E_ARG;
  try {
    return write_leaves(oct::refine_sharp_layer(base_level, max_level, centre, radius, alpha, tol), morton_out,
                        level_out, cap, n_out);
  } catch (...) {
    return GMG_E_OOM;
  }
}

gmg_status gmg_octree_balance(const uint64_t* morton, const uint8_t* level, int64_t n, uint64_t* morton_out,
                              uint8_t* level_out, int64_t cap, int64_t* n_out) {
  if (!morton || !level || n <= 0 || !n_out) return GMG_E_ARG;
  std::vector<oct::Leaf> t(static_cast<size_t>(n));
  for (int64_t i = 0; i < n; ++i) {
    if (morton[i] >> (3 * oct::kMaxLevel) || level[i] > oct::kMaxLevel) return GMG_E_MESH;
    uint32_t x, y, z;
    oct::morton_decode(morton[i], &x, &y, &z);
    t[i] = {static_cast<int32_t>(x), static_cast<int32_t>(y), static_cast<int32_t>(z), level[i]};
  }
  if (!oct::is_complete(t)) return GMG_E_MESH;
  try {
    return write_leaves(oct::balance(t), morton_out, level_out, cap, n_out);
  } catch (...) {
    return GMG_E_OOM;
  }
}

gmg_status gmg_level_leaves(const gmg_ctx* ctx, int32_t level, uint64_t* morton_out, uint8_t* level_out, int64_t cap,
                            int64_t* n_out) {
  if (!ctx || !n_out || check_level(ctx, level) != GMG_OK || !ctx->lv[level].oct) return GMG_E_ARG;
  return write_leaves(ctx->lv[level].leaves, morton_out, level_out, cap, n_out);
}

gmg_status gmg_num_elements(const gmg_ctx* ctx, int32_t level, int64_t* n) {
  if (!ctx || !n || check_level(ctx, level) != GMG_OK) return GMG_E_ARG;
  const Level& L = ctx->lv[level];
  *n = L.oct ? L.od.E : static_cast<int64_t>(L.n) * L.n * L.n;
  return GMG_OK;
}

gmg_status gmg_dof_coords(const gmg_ctx* ctx, int32_t level, double* xyz) {
  if (!ctx || !xyz || check_level(ctx, level) != GMG_OK) return GMG_E_ARG;
  const Level& L = ctx->lv[level];
  if (L.oct) {
    const double inv = 1.0 / static_cast<double>(oct::kTicks);
    for (int64_t k = 0; k < L.size; ++k) {
      const int64_t key = L.points[k];
      xyz[3 * k] = static_cast<double>(key % oct::kTicks) * inv;
      xyz[3 * k + 1] = static_cast<double>((key / oct::kTicks) % oct::kTicks) * inv;
      xyz[3 * k + 2] = static_cast<double>(key / (oct::kTicks * oct::kTicks)) * inv;
    }
    return GMG_OK;
  }
  std::vector<double> x(L.N);
  const std::vector<double> xi = lgl_nodes01(ctx->q);
  for (int i = 0; i < L.N; ++i) x[i] = (i / ctx->q + xi[i % ctx->q]) / L.n;
  for (int64_t k = 0; k < L.size; ++k) {
    xyz[3 * k] = x[k % L.N];
    xyz[3 * k + 1] = x[(k / L.N) % L.N];
    xyz[3 * k + 2] = x[k / (static_cast<int64_t>(L.N) * L.N)];
  }
  return GMG_OK;
}

gmg_status gmg_history(gmg_ctx* ctx, int32_t kind, double* out, int64_t cap, int64_t* count) {
  if (!ctx || !count || (kind != 0 && kind != 1) || cap < 0 || (cap > 0 && !out)) return GMG_E_ARG;
  const std::vector<double>& h = kind == 0 ? ctx->hist_res : ctx->hist_cyc;
  *count = static_cast<int64_t>(h.size());
  std::copy(h.begin(), h.begin() + std::min<int64_t>(cap, *count), out);
  return GMG_OK;
}

gmg_status gmg_timing_reset(gmg_ctx* ctx) {
  if (!ctx) return GMG_E_ARG;
  STCHK(drain_timing(ctx));
  std::fill(ctx->tsec.begin(), ctx->tsec.end(), 0.0);
  std::fill(ctx->tcount.begin(), ctx->tcount.end(), 0);
  return GMG_OK;
}

}  // extern "C"

namespace {

gmg_status ensure_net(gmg_ctx* c, int d) {
  NetDev& n = c->nets[d];
  if (n.w) return GMG_OK;
  STCHK(dalloc(c, reinterpret_cast<void**>(&n.w), sizeof(float) * kNetWeights));
  STCHK(dalloc(c, reinterpret_cast<void**>(&n.m), sizeof(float) * kNetWeights));
  STCHK(dalloc(c, reinterpret_cast<void**>(&n.v), sizeof(float) * kNetWeights));
  STCHK(dalloc(c, reinterpret_cast<void**>(&n.w1q), sizeof(float) * 432));
  STCHK(dalloc(c, reinterpret_cast<void**>(&n.w3q), sizeof(float) * 432));
  STCHK(dalloc(c, &n.w2fl, 16 * 15 * 64));
  STCHK(dalloc(c, &n.w2bl, 16 * 15 * 64));
  STCHK(dalloc(c, &n.w1l, 16 * 2 * 64));
  STCHK(dalloc(c, &n.w3l, 16 * 2 * 64));
  STCHK(dalloc(c, reinterpret_cast<void**>(&n.w2f), sizeof(uint16_t) * 6912));
  STCHK(dalloc(c, reinterpret_cast<void**>(&n.w2b), sizeof(uint16_t) * 6912));
  return GMG_OK;
}

// A depth that can hold a net (every level but the coarsest, which has no smoother)...
gmg_status check_net_depth(const gmg_ctx* c, int d) {
  if (!c || d < 0 || d >= c->L - 1) return GMG_E_ARG;
  return GMG_OK;
}

// ... and one whose level is a lattice of at least 16 nodes a side, where the net runs
gmg_status check_depth(const gmg_ctx* c, int d) {
  STCHK(check_net_depth(c, d));
  if (c->lv[c->L - 1 - d].latN < 16) return GMG_E_ARG;
  return GMG_OK;
}

// training (forward with its cache, backward, loss) runs on uniform meshes' levels
gmg_status check_train_depth(const gmg_ctx* c, int d) {
  STCHK(check_depth(c, d));
  if (c->lv[c->L - 1 - d].oct) return GMG_E_ARG;
  return GMG_OK;
}

gmg_status set_master(gmg_ctx* c, int d, const float* w_host) {
  STCHK(ensure_net(c, d));
  NetDev& n = c->nets[d];
  HIPCHK(c, hipMemcpyAsync(n.w, w_host, sizeof(float) * kNetWeights, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, launch_fill_zero(true, kNetWeights, n.m, c->stream));
  HIPCHK(c, launch_fill_zero(true, kNetWeights, n.v, c->stream));
  HIPCHK(c, launch_net_pack(n.w, n, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->net_set[d] = 1;
  // captured cycles bake in which levels use a net
  for (int k = 0; k < gmg_ctx::kGraphKeys; ++k)
    if (c->vgraph[k]) {
      (void)hipGraphExecDestroy(c->vgraph[k]);
      c->vgraph[k] = nullptr;
    }
  c->rho_plain = -1.0;
  return GMG_OK;
}

}  // namespace

extern "C" {

gmg_status gmg_net_cache_bytes(const gmg_ctx* ctx, int32_t depth, int64_t* bytes) {
  if (!bytes || check_depth(ctx, depth) != GMG_OK) return GMG_E_ARG;
  *bytes = net_cache_bytes(ctx->lv[ctx->L - 1 - depth].latN);
  return GMG_OK;
}

gmg_status gmg_net_set_weights(gmg_ctx* ctx, int32_t depth, const float* w_host, int64_t n) {
  if (!w_host || n != kNetWeights || check_net_depth(ctx, depth) != GMG_OK) return GMG_E_ARG;
  return scoped(ctx, [&] { return set_master(ctx, depth, w_host); });
}

gmg_status gmg_set_learned(gmg_ctx* ctx, int32_t depth, const uint16_t* w_bf16_host, int64_t n_w) {
  if (!w_bf16_host || n_w != kNetWeights || check_net_depth(ctx, depth) != GMG_OK) return GMG_E_ARG;
  std::vector<float> w(kNetWeights);
  for (int i = 0; i < kNetWeights; ++i) {
    const uint32_t u = static_cast<uint32_t>(w_bf16_host[i]) << 16;
    std::memcpy(&w[i], &u, sizeof(float));
  }
  return scoped(ctx, [&] { return set_master(ctx, depth, w.data()); });
}

gmg_status gmg_net_get_weights(gmg_ctx* ctx, int32_t depth, float* w_host, int64_t n) {
  if (!w_host || n != kNetWeights || check_net_depth(ctx, depth) != GMG_OK || !ctx->net_set[depth]) return GMG_E_ARG;
  return scoped(ctx, [&] {
    HIPCHK(ctx, hipMemcpyAsync(w_host, ctx->nets[depth].w, sizeof(float) * kNetWeights, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return GMG_OK;
  });
}

gmg_status gmg_net_get_state(gmg_ctx* ctx, int32_t depth, float* w_host, float* m_host, float* v_host) {
  if (!w_host || !m_host || !v_host || check_net_depth(ctx, depth) != GMG_OK || !ctx->net_set[depth]) return GMG_E_ARG;
  return scoped(ctx, [&] {
    const NetDev& n = ctx->nets[depth];
    const size_t bytes = sizeof(float) * kNetWeights;
    HIPCHK(ctx, hipMemcpyAsync(w_host, n.w, bytes, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(m_host, n.m, bytes, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(v_host, n.v, bytes, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return GMG_OK;
  });
}

gmg_status gmg_net_set_state(gmg_ctx* ctx, int32_t depth, const float* w_host, const float* m_host,
                             const float* v_host) {
  if (!w_host || !m_host || !v_host || check_net_depth(ctx, depth) != GMG_OK) return GMG_E_ARG;
  return scoped(ctx, [&] {
    STCHK(set_master(ctx, depth, w_host));
    const NetDev& n = ctx->nets[depth];
    const size_t bytes = sizeof(float) * kNetWeights;
    HIPCHK(ctx, hipMemcpyAsync(n.m, m_host, bytes, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(n.v, v_host, bytes, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return GMG_OK;
  });
}

gmg_status gmg_net_forward(gmg_ctx* ctx, int32_t depth, const float* x_dev, float* y_dev, void* cache_dev) {
  if (!x_dev || !y_dev || !cache_dev || check_train_depth(ctx, depth) != GMG_OK || !ctx->net_set[depth]) return GMG_E_ARG;
  const int N = ctx->lv[ctx->L - 1 - depth].N;
  return scoped(ctx, [&] {
    HIPCHK(ctx, launch_net_input(x_dev, nullptr, ctx->q, nullptr, ctx->part, ctx->part_cap, N, cache_dev, ctx->stream));
    HIPCHK(ctx, launch_net_forward(ctx->nets[depth], N, cache_dev, 0, nullptr, y_dev, ctx->stream));
    return GMG_OK;
  });
}

gmg_status gmg_net_backward(gmg_ctx* ctx, int32_t depth, const float* gy_dev, const void* cache_dev, float* gw_dev,
                            float* gin_dev) {
  if (!gy_dev || !cache_dev || !gw_dev || check_train_depth(ctx, depth) != GMG_OK || !ctx->net_set[depth])
    return GMG_E_ARG;
  const int N = ctx->lv[ctx->L - 1 - depth].N;
  const int64_t nv = static_cast<int64_t>(N) * N * N;
  if (ctx->g1g2_bytes < nv * 64) {
    STCHK(dalloc(ctx, &ctx->g1g2, static_cast<size_t>(nv * 64)));
    ctx->g1g2_bytes = nv * 64;
  }
  if (ctx->npart_floats < net_partial_floats(N)) {
    STCHK(dalloc(ctx, reinterpret_cast<void**>(&ctx->npart), sizeof(float) * net_partial_floats(N)));
    ctx->npart_floats = net_partial_floats(N);
  }
  return scoped(ctx, [&] {
    HIPCHK(ctx, launch_net_backward(ctx->nets[depth], N, cache_dev, gy_dev, ctx->g1g2, ctx->npart, gw_dev, gin_dev,
                                    ctx->stream));
    return GMG_OK;
  });
}

gmg_status gmg_adam_step(gmg_ctx* ctx, int32_t depth, const float* gw_dev, float lr, int64_t step) {
  if (!gw_dev || step < 1 || !(lr > 0.0f) || check_net_depth(ctx, depth) != GMG_OK || !ctx->net_set[depth])
    return GMG_E_ARG;
  return scoped(ctx, [&] {
    HIPCHK(ctx, launch_adam(ctx->nets[depth], gw_dev, lr, step, ctx->stream));
    return GMG_OK;
  });
}

gmg_status gmg_net_correction(gmg_ctx* ctx, int32_t level, const float* r_dev, float* e_dev) {
  if (!ctx || !r_dev || !e_dev || check_level(ctx, level) != GMG_OK || ctx->lv[level].latN < 16) return GMG_E_ARG;
  const int d = net_for_depth(ctx, ctx->L - 1 - level);
  if (d < 0) return fail(ctx, GMG_E_STATE, "no learned weights set");
  return scoped(ctx, [&] {
    STCHK(ensure_lcache(ctx, level));
    const Level& L = ctx->lv[level];
    HIPCHK(ctx, launch_fill_zero(true, L.size, e_dev, ctx->stream));
    HIPCHK(ctx, launch_net_input(r_dev, L.tab.stiff.dinv, ctx->q, ctx->scal + S_SSUM + level, ctx->part, ctx->part_cap, L.latN,
                                 ctx->lcache[level], ctx->stream));
    HIPCHK(ctx, launch_net_forward(ctx->nets[d], L.latN, ctx->lcache[level], 1, ctx->scal + S_SSUM + level, e_dev,
                                   ctx->stream, false));
    return GMG_OK;
  });
}

gmg_status gmg_residual(gmg_ctx* ctx, int32_t level, gmg_prec prec, const void* b_dev, const void* u_dev,
                        void* r_dev) {
  if (!ctx || !b_dev || !u_dev || !r_dev || u_dev == r_dev || check_level(ctx, level) != GMG_OK) return GMG_E_ARG;
  if (ctx->gen) STCHK(ensure_prec(ctx, pidx(prec)));  // the generic passes' temporaries
  return scoped(ctx, [&] { return apply_op(ctx, level, pidx(prec), Epi::Residual, u_dev, r_dev, b_dev, nullptr, 0, 0); });
}

gmg_status gmg_smooth_zero(gmg_ctx* ctx, int32_t level, gmg_prec prec, const void* b_dev, void* u_dev, int32_t nu) {
  if (!ctx || !b_dev || !u_dev || b_dev == u_dev || nu < 0 || check_level(ctx, level) != GMG_OK) return GMG_E_ARG;
  const int pi = pidx(prec);
  STCHK(ensure_prec(ctx, pi));
  return scoped(ctx, [&] { return smooth(ctx, level, pi, b_dev, u_dev, nu, true); });
}

gmg_status gmg_launch_shape(const gmg_ctx* ctx, int32_t level, gmg_prec prec, int32_t op, int32_t* shape_host) {
  if (!ctx || !shape_host || check_level(ctx, level) != GMG_OK || op < 0 || op > 5) return GMG_E_ARG;
  const Level& L = ctx->lv[level];
  const bool f32 = prec == GMG_FP32;
  for (int i = 0; i < 4; ++i) shape_host[i] = 0;
  if (L.oct || L.gen) {
    shape_host[0] = L.oct ? 5 : 6;
    return GMG_OK;
  }
  if (op >= 4) {
    if (level < 1) return GMG_E_ARG;
    const int Nc = ctx->lv[level - 1].N;
    const bool fused = !ctx->opt.no_fused_transfer &&
                       (op == 4 ? restrict_fusable(ctx->q, Nc) : prolong_fusable(ctx->q, Nc));
    shape_host[0] = fused ? 3 : 4;
    return GMG_OK;
  }
  static const Epi epis[4] = {Epi::Apply, Epi::Residual, Epi::Cheb, Epi::ChebZero};
  const ApplyShape sh = apply_shape(ctx->q, f32, epis[op], L.N, L.n, ctx->opt.q4_mfma != 0);
  if (sh.kernel < 0) return GMG_E_ARG;
  shape_host[0] = sh.kernel == 3 ? 7 : sh.kernel;
  shape_host[1] = sh.G;
  shape_host[2] = sh.TZ;
  shape_host[3] = sh.nblocks;
  return GMG_OK;
}

gmg_status gmg_net_loss_grad(gmg_ctx* ctx, int32_t depth, int32_t kind, const float* r_dev, const float* e_dev,
                             void* cache_dev, float* gw_dev, float scale, double* loss_host) {
  if (!r_dev || !cache_dev || !loss_host || check_train_depth(ctx, depth) != GMG_OK || !ctx->net_set[depth])
    return GMG_E_ARG;
  if (kind != 0 && kind != 1) return GMG_E_ARG;
  if (kind == 0 && !e_dev) return GMG_E_ARG;
  const int l = ctx->L - 1 - depth;
  STCHK(ensure_prec(ctx, 1));
  const int N = ctx->lv[l].N;
  const int64_t nv = ctx->lv[l].size;
  if (gw_dev) {
    if (ctx->g1g2_bytes < nv * 64) {
      STCHK(dalloc(ctx, &ctx->g1g2, static_cast<size_t>(nv * 64)));
      ctx->g1g2_bytes = nv * 64;
    }
    if (ctx->npart_floats < net_partial_floats(N)) {
      STCHK(dalloc(ctx, reinterpret_cast<void**>(&ctx->npart), sizeof(float) * net_partial_floats(N)));
      ctx->npart_floats = net_partial_floats(N);
    }
  }
  return scoped(ctx, [&] {
    Level& L = ctx->lv[l];
    const hipStream_t s = ctx->stream;
    float* y = static_cast<float*>(L.u[1]);
    float* et = static_cast<float*>(L.b[1]);
    float* d = static_cast<float*>(L.xp[1]);
    double* ssum = ctx->scal + S_SSUM + l;
    HIPCHK(ctx, launch_net_input(r_dev, L.tab.stiff.dinv, ctx->q, ssum, ctx->part, ctx->part_cap, N, cache_dev, s));
    HIPCHK(ctx, launch_net_forward(ctx->nets[depth], N, cache_dev, 0, nullptr, y, s));
    HIPCHK(ctx, launch_net_scale(y, ssum, nv, et, s));
    STCHK(apply_op(ctx, l, 1, Epi::Residual, et, d, r_dev, nullptr, 0, 0));  // d = r - A e~
    const float* gsrc = d;
    if (kind == 0) {
      // A e = r: ||e - e~||_A^2 = (e - e~)^T d and ||e||_A^2 = e^T r; dL/de~ = -2 d / e^T r
      HIPCHK(ctx, launch_dot(true, nv, e_dev, r_dev, ctx->part, ctx->scal + S_ER, s));
      HIPCHK(ctx, launch_dot(true, nv, e_dev, d, ctx->part, ctx->scal + S_ED, s));
      HIPCHK(ctx, launch_dot(true, nv, et, d, ctx->part, ctx->scal + S_TD, s));
    } else {
      // ||d||^2 / ||r||^2; dL/de~ = -2 A d / r^T r (A e~ no longer needed: reuse its buffer)
      HIPCHK(ctx, launch_dot(true, nv, r_dev, r_dev, ctx->part, ctx->scal + S_ER, s));
      HIPCHK(ctx, launch_dot(true, nv, d, d, ctx->part, ctx->scal + S_ED, s));
      if (gw_dev) {
        STCHK(apply_op(ctx, l, 1, Epi::Apply, d, et, nullptr, nullptr, 0, 0));
        gsrc = et;
      }
    }
    if (gw_dev) {
      HIPCHK(ctx, launch_net_loss_gy(gsrc, ssum, ctx->scal + S_ER, static_cast<double>(scale), nv, y, s));
      HIPCHK(ctx, launch_net_backward(ctx->nets[depth], N, cache_dev, y, ctx->g1g2, ctx->npart, gw_dev, nullptr, s));
    }
    double hs[kNumScal];
    STCHK(read_scalars(ctx, hs, kNumScal));
    *loss_host = kind == 0 ? (hs[S_ED] - hs[S_TD]) / hs[S_ER] : hs[S_ED] / hs[S_ER];
    return GMG_OK;
  });
}

gmg_status gmg_solve(gmg_ctx* ctx, const double* f_dev, double* u_dev, double rtol, gmg_info* info) {
  if (!ctx || !f_dev || !u_dev) return GMG_E_ARG;
  if (!ctx->bint) STCHK(dalloc(ctx, &ctx->bint, sizeof(double) * ctx->lv.back().size));
  STCHK(gmg_rhs(ctx, f_dev, static_cast<double*>(ctx->bint)));
  return gmg_solve_rhs(ctx, static_cast<const double*>(ctx->bint), u_dev, rtol, info);
}

}  // extern "C"
