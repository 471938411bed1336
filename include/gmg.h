/*
 * gmg.h -- C ABI of the MI355X geometric-multigrid library (libgmg.so).
 *
 * The library solves the periodic Poisson problem -Laplace(u) = f on the unit
 * cube (eq. 1.1 of Gholami, Malhotra, Sundar, Biros, "FFT, FMM, or Multigrid?")
 * with continuous Galerkin Q_q elements on LGL nodes (Section 2.3.2), a
 * multigrid hierarchy of nested meshes (Section 2.3.1), a Chebyshev-accelerated
 * Jacobi smoother (Section 2.3.3), P(i,j) = phi_j^{k-1}(p_i) and R = P^T
 * (Section 2.3.4, eqs. 2.1-2.2), the V-cycle of Algorithm 2.1 with a direct
 * coarsest solve, and CG preconditioned by one V-cycle (Section 2.3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every call returns a gmg_status; nothing throws across the ABI.
 *  - Pointers named *_dev are device pointers (HIP global memory) owned by the
 *    caller; the library never frees them.  Pointers named *_host are host
 *    memory.  The library owns the context and every buffer inside it.
 *  - Vectors are DoF vectors of one level.  Uniform meshes: length N^3 with
 *    N = q * n_level, lexicographic with x fastest: index i + N (j + N k); lattice
 *    node i sits at x = (e + xi_a) / n_level, e = i div q, a = i mod q, xi the LGL
 *    nodes on [0,1].  Octree meshes: the independent nodes (hanging nodes are not
 *    DoFs) in ascending order of x + T (y + T z), with (x, y, z) the node position
 *    in units of 2^-11 and T = 2^11 (gmg_dof_coords returns the positions); for
 *    an octree whose leaves all have one level this is the uniform order.
 *  - A vector's element type is double for GMG_FP64 and float for GMG_FP32.
 *  - Calls are ordered on the HIP stream given to gmg_setup: the library runs
 *    its kernels on a stream of its own after the work already queued there,
 *    and the caller's stream waits for them.  gmg_apply,
 *    gmg_smooth, gmg_restrict, gmg_prolong, gmg_coarse_solve, gmg_vcycle and
 *    gmg_rhs enqueue work and return without synchronizing.  gmg_solve,
 *    gmg_dot and the query calls synchronize the stream.
 *  - Input and output device buffers of one call must not overlap unless the
 *    call says so.
 *  - A context is not thread-safe; distinct contexts are independent.
 *  - Errors: GMG_E_ARG for an invalid argument (null pointer, level out of
 *    range, order not in {1, ..., 8}, n not a power of two, ...); GMG_E_HIP when a
 *    HIP runtime call fails (the context should then be destroyed);
 *    GMG_E_NOCONV when a solve stops at max_iters (info is filled);
 *    GMG_E_BREAKDOWN for NaN/Inf or a non-positive p^T A p; GMG_E_OOM when a
 *    device allocation fails.  gmg_last_error() returns a message for the last
 *    failing call on a context.
 */
#ifndef GMG_H
#define GMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gmg_ctx gmg_ctx;

typedef enum {
  GMG_OK = 0,
  GMG_E_ARG = 1,
  GMG_E_MESH = 2,
  GMG_E_OOM = 3,
  GMG_E_HIP = 4,
  GMG_E_NOCONV = 5,
  GMG_E_BREAKDOWN = 6,
  GMG_E_STATE = 7
} gmg_status;

typedef enum { GMG_FP64 = 0, GMG_FP32 = 1 } gmg_prec;

/* Mesh description.  Uniform periodic meshes: n = elements per direction, a power
 * of two with q*n >= 4, and order q in {1, ..., 8} (Section 2.3.2 admits up to 16).
 * Orders 1, 2, 4 run the specialised streaming kernels, 2 <= n <= 512 (256 for q = 4);
 * orders 3, 5, 6, 7, 8 run generic kernels (three banded passes per operator apply,
 * one-axis transfer passes), 1 <= n <= 64, and their hierarchies may end on a single
 * periodic element (n = 1, where coarsening ends, Section 2.3.1).
 * levels = number of multigrid levels (level 0 coarsest, levels-1 finest, n
 * halves per level, Section 2.3.1); 0 selects the deepest hierarchy whose
 * coarsest level has at most 512 DoFs and at least 2 elements per direction (1 for
 * the generic orders).
 * The coarsest level is solved with a dense FP64 pseudo-inverse, so an explicit
 * `levels` must leave at most 512 DoFs there (else GMG_E_ARG).
 *
 * Octree meshes (n = 0; order 1 or 2): a complete, 2:1-balanced linear octree
 * of the periodic unit cube (Sections 2.2.1 and 2.3.1), given as n_leaves leaves
 * sorted by Morton key: leaf_morton[i] interleaves the bits of the leaf's anchor
 * (x, y, z) in units of 2^-10 (x in the lowest bit of each triple) and
 * leaf_level[i] in [2, 10] is its level (width 2^-level).  Balance is across
 * faces, edges and corners, wrapping periodically.  The hierarchy coarsens by
 * merging every complete family of 8 sibling leaves and balancing again
 * (Section 2.3.1) until the mesh is uniform at level 2; levels > 0 keeps the
 * finest `levels` meshes of that sequence.  Host arrays, read during
 * gmg_setup only.  An unsorted, incomplete or unbalanced octree gives GMG_E_MESH. */
typedef struct {
  int32_t order;
  int32_t n;              /* elements per direction; 0 for an octree mesh       */
  int32_t levels;
  int32_t reserved;
  int64_t n_leaves;       /* octree meshes only                                  */
  const uint64_t* leaf_morton;
  const uint8_t* leaf_level;
} gmg_mesh;

/* Solver options.  Zero-initialized fields take the defaults given here. */
typedef struct {
  int32_t cheb_degree;      /* Chebyshev polynomial degree (default 3)                    */
  int32_t nu_pre, nu_post;  /* polynomial applications before/after correction (2, 2)      */
  double cheb_lo, cheb_hi;  /* [alpha, beta] = [lo, hi] * lambda_hat (0.1, 1.1)            */
  int32_t lanczos_steps;    /* Lanczos steps for lambda_hat of D^-1 A (10; Section 2.3.3)  */
  int32_t smoother;         /* 0 Chebyshev-Jacobi, 1 damped Jacobi (omega below)           */
  double jacobi_omega;      /* damping of the Jacobi smoother (2/3)                        */
  uint64_t seed;            /* key of the SplitMix64 Lanczos start vectors (0)             */
  int32_t vcycle_prec;      /* GMG_FP64: CG on FP64 V-cycles.  GMG_FP32: FP32 V-cycles
                               with FP64 refinement, as chosen by ir_mode               */
  int32_t krylov;           /* 0 PCG, 1 FCG(1) (forced to 1 with FP32 V-cycles)            */
  double inner_rtol;        /* floor of the inner FP32 relative tolerance (2e-6)           */
  int32_t max_iters;        /* cap on Krylov iterations, inner+outer (500)                 */
  double lambda_override;   /* > 0: use this lambda_hat on every level instead of Lanczos  */
  int32_t timing;           /* != 0: bracket every operator-apply launch with HIP events
                               (read back with gmg_timing_get); disables graph replay      */
  int32_t no_graphs;        /* != 0: launch the V-cycles of gmg_solve eagerly instead of
                               replaying the HIP graph captured on first use               */
  int32_t ir_mode;          /* FP32 V-cycles only.  0: FP64 flexible CG whose preconditioner
                               is one FP32 V-cycle (FP64 residual, update, dots and
                               projection at every iteration).  1: nested refinement,
                               FP64 residual / update around FP32 flexible CG solves    */
  int32_t use_learned;      /* != 0: learned smoother in every smoothing phase of levels with
                               at least 16 lattice nodes per direction (forces FP32
                               V-cycles and flexible CG); see gmg_set_learned            */
  int32_t learned_depths;   /* > 0: only depths 0 .. learned_depths-1 use a net; the other
                               levels keep the Chebyshev smoother (0: every level)       */
  int32_t no_fused_tail;    /* != 0: run the level of 16^3 nodes next to the coarsest with
                               the separate kernels of every other level instead of the
                               one-workgroup kernels that keep it in LDS (testing aid)  */
  int32_t learned_min_depth; /* > 0: depths below this keep the Chebyshev smoother (the
                               finest levels, where a net application costs the most)   */
  int32_t no_speculation;   /* != 0: FP64 flexible CG around FP32 V-cycles waits for each
                               residual norm before it enqueues the next V-cycle, instead
                               of enqueueing it while the norm is read back whenever the
                               last norm was far above the tolerance (testing aid)      */
  int32_t no_fused_transfer; /* != 0: restrict and prolong on uniform levels with three
                               one-axis passes instead of the one-pass kernels (the same
                               bits; testing aid)                                        */
  int32_t no_fused_test_norms; /* != 0: the test of a learned cycle stores the residual and
                               reduces the two norms in a pass of its own instead of in the
                               residual's epilogue (the same norms up to summation order;
                               testing aid)                                              */
  int32_t q4_mfma;          /* != 0: the FP32 q = 4 applies, residuals and smoother steps on
                               uniform levels of N >= 64 nodes take the x and z passes of
                               the sum factorization (Section 4: 1D contractions of the
                               element-local values) on the matrix cores (4x4x1 FP32
                               MFMA) instead of the vector unit; the same operator to FP32
                               rounding.  Off by default: measured slower here (the vector
                               form is not bound by its arithmetic)                       */
} gmg_options;

typedef struct {
  int32_t outer_iters;      /* iterative-refinement steps (0 for plain FP64 PCG)           */
  int32_t inner_iters;      /* total Krylov iterations                                     */
  int32_t fallbacks;        /* learned cycles replaced by the plain cycle                  */
  int32_t reserved;
  double rel_residual_f64;  /* final ||b - A u||_2 / ||b||_2, recomputed in FP64           */
  double t_setup;           /* seconds spent in gmg_setup (host clock)                     */
  double t_solve;           /* seconds inside the solve (HIP events on the stream)         */
  /* per-phase seconds of the solve (Section 3's Setup / Eval / Comm split, taken down to
   * the V-cycle phases); filled only with gmg_options.timing != 0, else 0:            */
  double t_smooth;          /* smoother steps, every level and precision                  */
  double t_transfer;        /* restriction and prolongation                               */
  double t_coarse;          /* coarsest solve                                             */
  double t_learned;         /* learned corrections (residual, input scaling, net)         */
} gmg_info;

/* Build the hierarchy on the current HIP device: operator tables, diagonal
 * (Section 2.3, Setup), Lanczos estimate of lambda_max(D^-1 A) per level
 * (Section 2.3.3), coarsest-level pseudo-inverse (dense FP64), device buffers.
 * hip_stream: a hipStream_t (NULL = the null stream).  *out receives the context. */
gmg_status gmg_setup(const gmg_mesh* mesh, const gmg_options* opts, void* hip_stream, gmg_ctx** out);
gmg_status gmg_destroy(gmg_ctx* ctx);

/* Queries (host).  gmg_dof_coords_1d writes the N coordinates of one axis of a
 * uniform mesh (GMG_E_ARG on octree meshes); the DoF (i, j, k) sits at
 * (x[i], x[j], x[k]). */
gmg_status gmg_num_levels(const gmg_ctx* ctx, int32_t* levels);
gmg_status gmg_num_dofs(const gmg_ctx* ctx, int32_t level, int64_t* n);
gmg_status gmg_dof_coords_1d(const gmg_ctx* ctx, int32_t level, double* x_host);
gmg_status gmg_lambda(const gmg_ctx* ctx, int32_t level, double* lambda_host);

/* d_dev[i] = A_ii on a level (FP64), the Jacobi diagonal of Section 2.3 Setup. */
gmg_status gmg_diagonal(gmg_ctx* ctx, int32_t level, double* d_dev);

/* y = A_level x: matrix-free, sum-factorized stiffness apply (Section 2.3.2). */
gmg_status gmg_apply(gmg_ctx* ctx, int32_t level, gmg_prec prec, const void* x_dev, void* y_dev);

/* y = M_level x with the consistent mass matrix of the continuous Galerkin LGL
 * discretization (Sections 2.3 and 2.3.2): the same sum-factorized kernel with the 1D
 * mass rows in every direction.  It forms the load vector of the discrete system
 * A_h u_h = f_h from nodal source values (gmg_rhs). */
gmg_status gmg_mass(gmg_ctx* ctx, int32_t level, gmg_prec prec, const void* x_dev, void* y_dev);

/* u <- S^nu (u; b): nu applications of the level smoother to A u = b, in place
 * (Section 2.3.3).  u_dev holds the initial guess on entry. */
gmg_status gmg_smooth(gmg_ctx* ctx, int32_t level, gmg_prec prec, const void* b_dev, void* u_dev, int32_t nu);

/* rc = R rf = P^T rf from level `level` (fine) to level-1 (Section 2.3.4). */
gmg_status gmg_restrict(gmg_ctx* ctx, int32_t level, gmg_prec prec, const void* rf_dev, void* rc_dev);

/* uf += P ec from level-1 to level `level` (eq. 2.2). */
gmg_status gmg_prolong(gmg_ctx* ctx, int32_t level, gmg_prec prec, const void* ec_dev, void* uf_dev);

/* x = A_0^+ (b - mean(b)) on the coarsest level, computed in FP64 whatever prec
 * says (the direct coarsest solve of Algorithm 2.1). */
gmg_status gmg_coarse_solve(gmg_ctx* ctx, gmg_prec prec, const void* b_dev, void* x_dev);

/* z = V r: one V-cycle (Algorithm 2.1) on the finest level, zero initial guess. */
gmg_status gmg_vcycle(gmg_ctx* ctx, gmg_prec prec, const void* r_dev, void* z_dev);

/* r = b - A_level u (vectors of type prec): the residual step of Algorithm 2.1 on one
 * level, in the same fused kernel as the apply. */
gmg_status gmg_residual(gmg_ctx* ctx, int32_t level, gmg_prec prec, const void* b_dev, const void* u_dev, void* r_dev);

/* u = S^nu (0; b): nu applications of the level smoother from a zero initial guess,
 * the pre-smoothing of Algorithm 2.1 (Section 2.3.3).  u_dev need not be initialized
 * and must not alias b_dev.  On uniform levels with a Chebyshev smoother the first
 * two steps run as one pass that forms x_1 = D^-1 b / theta as it loads b. */
gmg_status gmg_smooth_zero(gmg_ctx* ctx, int32_t level, gmg_prec prec, const void* b_dev, void* u_dev, int32_t nu);

/* Launch shape of one operation on a level (a tracing aid: which kernel instance the
 * calls above launch there).  op: 0 y = A x, 1 r = b - A x, 2 smoother step, 3 the
 * fused first two smoother steps from a zero guess, 4 restriction onto level-1,
 * 5 prolongation from level-1.  shape_host[0..3] (host, 4 values):
 *   [0] kernel: 0 point kernel (one thread per element column, levels of N <= 32
 *       nodes), 1 streaming column kernel, 2 column kernel that loads all planes of its
 *       one-layer z chunk at once, 3 one-pass (fused) transfer, 4 three one-axis
 *       transfer passes, 5 octree kernels, 6 generic-order kernels, 7 streaming
 *       column kernel with its x and z passes on the matrix cores (option q4_mfma);
 *   [1] G (a tile is 4G lattice rows), [2] TZ (element layers per block; 0 for the
 *   point kernel), [3] blocks per launch (0 for transfers and octree levels).
 * GMG_E_ARG for an invalid level or op (restriction and prolongation need level >= 1). */
gmg_status gmg_launch_shape(const gmg_ctx* ctx, int32_t level, gmg_prec prec, int32_t op, int32_t* shape_host);

/* b = M f - mean(M f): load vector of nodal source values f on the finest level, the
 * right-hand side f_h of the Galerkin system A_h u_h = f_h (Section 2.3) for a source
 * interpolated in the LGL nodal basis (Section 2.3.2).  The mean is removed because on
 * the periodic unit cube (Section 1, limitations) the system is solvable only for a
 * right-hand side orthogonal to the constants. */
gmg_status gmg_rhs(gmg_ctx* ctx, const double* f_dev, double* b_dev);

/* Solve A u = b(f) to ||b - A u||_2 <= rtol ||b||_2 (true FP64 residual); u is
 * returned with zero integral.  f_dev: nodal source values (FP64).  The
 * variant gmg_solve_rhs takes an already projected load vector b_dev. */
gmg_status gmg_solve(gmg_ctx* ctx, const double* f_dev, double* u_dev, double rtol, gmg_info* info);
gmg_status gmg_solve_rhs(gmg_ctx* ctx, const double* b_dev, double* u_dev, double rtol, gmg_info* info);

/* Exact solve of the same finite-element system by the 3D FFT (the FFT Poisson method of
 * Section 2, Table 7's uniform-grid baseline), for uniform meshes of every order.  Q1: on a
 * periodic mesh the Q1 matrix is diagonal in the Fourier basis, with eigenvalue
 *   kap(kx) mu(ky) mu(kz) + mu(kx) kap(ky) mu(kz) + mu(kx) mu(ky) kap(kz),
 *   kap(k) = (2 - 2 cos(2 pi k/N)) / h,  mu(k) = h (4 + 2 cos(2 pi k/N)) / 6,
 * so u = F^-1 [F(b) / eigenvalue] with the constant mode set to zero (the zero-integral
 * solution).  Q2, Q4: the q^3 node classes make the matrix block-circulant over the
 * elements; per wavenumber the q^3 x q^3 symbol is the Kronecker sum of the 1D q x q
 * symbols, inverted in the eigenbasis of each axis's q x q pencil (K, M), with the
 * constant mode (the integral) set to zero.  b_dev: the load vector (as for gmg_solve_rhs, mean zero), u_dev: the
 * solution, both FP64 device arrays of gmg_num_dofs values in lattice order, not
 * aliased; b_dev is not modified.  FP64 transforms (hipFFT).  The first call allocates
 * the transform plans and a spectrum buffer of N^2 (N/2+1) complex values, kept until
 * gmg_destroy (Q2, Q4: q^3 class spectra and class arrays).  GMG_E_ARG on octree contexts
 * and on aliasing. */
gmg_status gmg_fft_solve(gmg_ctx* ctx, const double* b_dev, double* u_dev);

/* The paper's FFT Poisson method (Section 2.1, last paragraph): the spectral solution of
 * -Laplace(u) = f on the uniform grid x = (i, j, k) / N of the periodic unit cube: the 3D
 * discrete Fourier transform of f, each coefficient divided by 4 pi^2 |m|^2 (m the integer
 * wavevector, components in {-N/2 .. N/2-1}; the m = 0 coefficient, the mean, set to 0),
 * the inverse transform.  u is the zero-mean solution; the mean of f is ignored.
 * gmg_spectral_create: N a power of two, 16 <= N <= 1024 (else GMG_E_ARG); allocates a
 * complex FP64 work buffer of N^3 values (16 N^3 bytes) and a table of N roots of unity,
 * kept until gmg_spectral_destroy; hip_stream: a hipStream_t (NULL = the null stream) on
 * which gmg_spectral_solve enqueues its five kernels (hand-written transforms, no FFT
 * library) and returns without synchronizing.  f_dev, u_dev: N^3 FP64 device values, x
 * fastest (index i + N (j + N k)), caller-owned; they may alias.  A solver object is not
 * thread-safe and must not run two solves at once. */
typedef struct gmg_spectral gmg_spectral;
gmg_status gmg_spectral_create(int32_t N, void* hip_stream, gmg_spectral** out);
gmg_status gmg_spectral_solve(gmg_spectral* sp, const double* f_dev, double* u_dev);
gmg_status gmg_spectral_destroy(gmg_spectral* sp);

/* *out_host = sum_i x_i y_i accumulated in FP64 (x, y of type prec, length n): the inner
 * products of the conjugate gradient iteration that the V-cycle preconditions (Section
 * 2.3), in a fixed summation order (block partials, then one pass over them). */
gmg_status gmg_dot(gmg_ctx* ctx, gmg_prec prec, int64_t n, const void* x_dev, const void* y_dev, double* out_host);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): gmg_dot without any allocation and
 * without synchronizing.  *out_dev (one double of device memory owned by the caller) =
 * sum_i x_i y_i accumulated in FP64, the same kernels and summation order as gmg_dot (so
 * the same bits); x_dev, y_dev: n values of type prec.  Enqueued in the stream order of
 * the other enqueue-only calls; read *out_dev after synchronizing the caller's stream.
 * The partials of the first pass go to a static device array of 1024 FP64 values
 * (8 KiB per device, held until the process ends, its address looked up once per device
 * in gmg_setup); the first pass uses at most 1024 blocks whatever n is, so every n >= 0
 * fits (GMG_E_ARG if the block count ever exceeded the array).  Every call on one device
 * shares that array and leaves its partials there: calls that overlap on one device (on
 * different streams or contexts) race.  Calls no hipMalloc, hipFree or allocating
 * library routine.  n = 0 writes 0 (x_dev and y_dev may then be null).  GMG_E_ARG for
 * null pointers, n < 0 or a current device other than the context's; GMG_E_STATE if the
 * array's address was not set up on this device. */
gmg_status gmg_dot_noalloc(gmg_ctx* ctx, gmg_prec prec, int64_t n, const void* x_dev, const void* y_dev,
                           double* out_dev);

/* ---------------------------------------------------------------------------
 * Learned smoother (not in the paper, whose smoother choice is heuristic, Section 1
 * "Limitations" and Section 2.3.3).  One net per depth d (d = 0 finest level,
 * d = levels-2 the level above the coarsest); a depth without weights uses the
 * deepest depth that has them.  Net: Conv3d(1->16) - ReLU - Conv3d(16->16) - ReLU -
 * Conv3d(16->1), 3x3x3, circular padding on the level's DoF lattice, no bias,
 * BF16 weights and activations, FP32 accumulation.  Weights are 7776 values in
 * the flat layout W1[co][t] (432), W2[co][ci][t] (6912), W3[ci][t] (432), tap
 * t = (dz+1)*9 + (dy+1)*3 + (dx+1), out(v) = sum_t W[.., t] in(v + (dx, dy, dz)).
 * In a learned cycle each smoothing phase is (nu - 1) Chebyshev applications then
 * u <- u + s N(D^-1 (b - A u) / s), s = RMS(D^-1 (b - A u)).  Inside gmg_solve each
 * learned cycle is kept only if ||r - A z|| / ||r|| is no larger than the plain
 * cycle's last measured value (initialized by two plain cycles on a seeded
 * vector); otherwise the plain FP32 cycle replaces it (info->fallbacks).
 * The lattice must have at least 16 nodes per direction (GMG_E_ARG otherwise).  On an
 * octree hierarchy the levels whose leaves all have one level are uniform lattices (their
 * DoFs are numbered in lattice order) and take the net like uniform levels; the adaptive
 * levels keep the polynomial smoother (a lattice convolution is undefined across leaf sizes).
 * ------------------------------------------------------------------------- */

/* FP32 master weights of one depth (host, 7776 values); resets its Adam state. */
gmg_status gmg_net_set_weights(gmg_ctx* ctx, int32_t depth, const float* w_host, int64_t n);
/* BF16 weights (host, 7776 values, round-to-nearest-even bit patterns) of one depth. */
gmg_status gmg_set_learned(gmg_ctx* ctx, int32_t depth, const uint16_t* w_bf16_host, int64_t n_w);
gmg_status gmg_net_get_weights(gmg_ctx* ctx, int32_t depth, float* w_host, int64_t n);
/* Bytes of the activation cache of gmg_net_forward / gmg_net_backward at one depth. */
gmg_status gmg_net_cache_bytes(const gmg_ctx* ctx, int32_t depth, int64_t* bytes);
/* y = N_depth(x) on the depth's lattice (x, y FP32 device vectors); cache_dev
 * (caller-owned, gmg_net_cache_bytes) receives bf16(x) and both activations. */
gmg_status gmg_net_forward(gmg_ctx* ctx, int32_t depth, const float* x_dev, float* y_dev, void* cache_dev);
/* Training state of one depth for checkpoints (host FP32 arrays of 7776 values each):
 * the master weights and Adam's first and second moment estimates.  gmg_net_set_state
 * installs all three (and re-rounds the BF16 copies); gmg_adam_step then continues
 * from them with the caller's step count. */
gmg_status gmg_net_get_state(gmg_ctx* ctx, int32_t depth, float* w_host, float* m_host, float* v_host);
gmg_status gmg_net_set_state(gmg_ctx* ctx, int32_t depth, const float* w_host, const float* m_host,
                             const float* v_host);
/* gw_dev (7776 FP32, device) += d(sum gy . y)/dw for the forward pass held in
 * cache_dev; gin_dev (may be NULL) = d(sum gy . y)/d bf16(x). */
gmg_status gmg_net_backward(gmg_ctx* ctx, int32_t depth, const float* gy_dev, const void* cache_dev, float* gw_dev,
                            float* gin_dev);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; step counts from 1) on the FP32
 * master weights of one depth, then re-rounds the BF16 copies. */
gmg_status gmg_adam_step(gmg_ctx* ctx, int32_t depth, const float* gw_dev, float lr, int64_t step);
/* Training loss of one pair on the depth's level (FP32 device vectors), with
 * e~ = s N(D^-1 r / s), returned in *loss_host:
 *   kind 0 (energy)    ||e - e~||_A^2 / ||e||_A^2 for e = A^+ r, evaluated as
 *                      (e - e~)^T (r - A e~) / (e^T r);
 *   kind 1 (residual)  ||r - A e~||_2^2 / ||r||_2^2 (e_dev unused, may be NULL).
 * If gw_dev is not NULL, gw_dev += scale * d loss / dw (backward through A and the
 * net).  The level's FP32 work vectors are overwritten. */
gmg_status gmg_net_loss_grad(gmg_ctx* ctx, int32_t depth, int32_t kind, const float* r_dev, const float* e_dev,
                             void* cache_dev, float* gw_dev, float scale, double* loss_host);
/* e = s N(D^-1 r / s) on one level (FP32 device vectors): the learned correction. */
gmg_status gmg_net_correction(gmg_ctx* ctx, int32_t level, const float* r_dev, float* e_dev);

/* Per-kernel timing, a tracing aid (Section 3 reports Setup/Eval/Comm phase
 * times; this goes down to single launches).  With gmg_options.timing != 0,
 * every launch of the operator-apply kernel is bracketed by HIP events on the
 * context stream; inside a smoothing phase the consecutive steps of kinds 2 and
 * 3 on one level are bracketed as one run, whose time is split between the two
 * kinds in proportion to their traffic (3 : 4 per launch), so that the events'
 * own dispatch time is not added to each step.  gmg_timing_get synchronizes
 * the stream and returns, for one level, kind and precision, the number of
 * launches and their summed duration in seconds since setup or the last
 * gmg_timing_reset.  Kinds:
 *   0 y = A x            (algorithmic traffic 2 values per DoF)
 *   1 r = b - A x        (3 values per DoF)
 *   2 smoother step without a previous iterate, x' = x + c D^-1 (b - A x)
 *                        (3 values per DoF)
 *   3 smoother step x' = x + c1 (x - x_prev) + c2 D^-1 (b - A x)
 *                        (4 values per DoF)
 *   4 y = M x            (2 values per DoF)
 * and, bracketing a whole step (all its launches):
 *   5 restriction to this level's coarser neighbour   6 prolongation from it
 *   7 coarsest solve (level 0)                        8 learned correction
 *   9 first smoother step from a zero guess, x = c D^-1 b (2 values per DoF; octree
 *     levels and degree-1 smoothers)
 *  10 first two Chebyshev steps from a zero guess in one pass on uniform levels:
 *     x_1 = D^-1 b / theta formed from b as it is loaded, x_2 = x_1 + c1 x_1 +
 *     c2 D^-1 (b - A x_1); x_1 and x_2 are stored (3 values per DoF)
 *  11 the cycle of the uniform 16^3-node level next to the coarsest, run by one
 *     workgroup from LDS (pre-smoothing, residual and restriction; prolongation
 *     and post-smoothing: two launches per cycle)                               */
gmg_status gmg_timing_get(gmg_ctx* ctx, int32_t level, int32_t kind, gmg_prec prec, int64_t* launches,
                          double* seconds);
gmg_status gmg_timing_reset(gmg_ctx* ctx);

/* Octree construction (host, integer work; Section 2.3.1, refinement on the
 * gradient of f as in Section 3).  Outputs are leaves in the gmg_mesh format;
 * cap is the capacity of the output arrays and *n_out receives the number of
 * leaves (when it exceeds cap, nothing is written and GMG_E_ARG is returned).
 *
 * gmg_octree_refine_gaussians: start from the uniform mesh of base_level, split
 * every leaf O with level < max_level and
 *     h_O sum_i |a_i| g_i(d_i) > tol sum_i |a_i|,
 * d_i = periodic distance from centre i to the box of O,
 * g_i(d) = (d' / s_i^2) exp(-d'^2 / (2 s_i^2)), d' = max(d, s_i) (a bound on the
 * gradient of a_i exp(-r^2 / (2 s_i^2)) over the box), until no leaf is split;
 * then 2:1 balance.  centres: 3 * count doubles (x, y, z), sigma, amps: count.
 * gmg_octree_refine_sharp_layer: the same for f = -Laplace(u) of the sharp-layer
 * solution u = exp(-(r/R)^alpha) of the paper's second time-to-solution test
 * (Section 3), r the periodic distance to centre (3 doubles in [0, 1)): split
 * while h_O max|f'| > tol max|f|, the maxima from a radial table with spacing
 * R / (16 alpha) over the entries that cover O's distance range from the centre.
 * R > 0, 2 < alpha <= 1e4.
 * gmg_octree_balance: the coarsest 2:1-balanced refinement of a complete octree
 * (GMG_E_MESH if the input is not complete).
 * gmg_level_leaves: the leaves of one level of an octree context.
 * gmg_num_elements: elements of one level (uniform: n_level^3). */
gmg_status gmg_octree_refine_gaussians(int32_t base_level, int32_t max_level, int32_t count, const double* centres_host,
                                       const double* sigma_host, const double* amps_host, double tol,
                                       uint64_t* morton_out, uint8_t* level_out, int64_t cap, int64_t* n_out);
gmg_status gmg_octree_refine_sharp_layer(int32_t base_level, int32_t max_level, const double* centre_host,
                                         double radius, double alpha, double tol, uint64_t* morton_out,
                                         uint8_t* level_out, int64_t cap, int64_t* n_out);
gmg_status gmg_octree_balance(const uint64_t* morton_host, const uint8_t* level_host, int64_t n, uint64_t* morton_out,
                              uint8_t* level_out, int64_t cap, int64_t* n_out);
gmg_status gmg_level_leaves(const gmg_ctx* ctx, int32_t level, uint64_t* morton_out, uint8_t* level_out, int64_t cap,
                            int64_t* n_out);
gmg_status gmg_num_elements(const gmg_ctx* ctx, int32_t level, int64_t* n);

/* Coordinates of every DoF of a level (uniform or octree): xyz_host[3 k + d] is
 * coordinate d of DoF k, in [0, 1). */
gmg_status gmg_dof_coords(const gmg_ctx* ctx, int32_t level, double* xyz_host);

/* Convergence history of the last gmg_solve / gmg_solve_rhs (Section 3 reports
 * iteration counts; this keeps every iterate).  Host call, no synchronization.
 *   kind 0: the Krylov residual norm ||r_k||_2 at every iteration, starting with
 *           the initial one, in the order the Krylov loops ran (with nested
 *           refinement the inner FP32 solves follow each other).
 *   kind 1: one triple per learned-cycle test: the learned cycle's contraction
 *           rho_L = ||r - A z_L|| / ||r||, the reference contraction it was compared
 *           with, and the plain cycle's contraction on the same r when the learned
 *           cycle was rejected (NaN when it was kept).
 * *count receives the number of values recorded; min(cap, *count) of them are
 * copied to out (host memory owned by the caller; may be NULL when cap is 0). */
gmg_status gmg_history(gmg_ctx* ctx, int32_t kind, double* out_host, int64_t cap, int64_t* count);

const char* gmg_status_string(gmg_status s);
const char* gmg_last_error(const gmg_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* GMG_H */
