// Host-side octree meshing of the library: the periodic linear octree, its 2:1
// balance and coarsening (Section 2.3.1), and the continuous Q_q element space
// with hanging nodes on it (Section 2.3; hanging nodes, Section 4).
#pragma once

#include <cstdint>
#include <vector>

namespace gmg {
namespace oct {

constexpr int kMaxLevel = 10;              // finest leaf level
constexpr int32_t kUnits = 1 << kMaxLevel; // leaf anchors in units of 2^-kMaxLevel
constexpr int64_t kTicks = 2 * kUnits;     // node positions in units of 2^-(kMaxLevel+1)

struct Leaf {
  int32_t x, y, z;  // anchor, in units
  int32_t level;
};

inline int32_t leaf_size(int level) { return 1 << (kMaxLevel - level); }

// Bits of x, y, z interleaved, x in the lowest bit of each triple.
uint64_t morton_key(uint32_t x, uint32_t y, uint32_t z);
void morton_decode(uint64_t key, uint32_t* x, uint32_t* y, uint32_t* z);

// Sorted by Morton key, aligned, Morton ranges contiguous, covering the cube.
bool is_complete(const std::vector<Leaf>& t);
// No two touching leaves (faces, edges, corners; periodic) differ by more than one level.
bool is_balanced(const std::vector<Leaf>& t);
// The coarsest 2:1-balanced refinement of a complete octree.
std::vector<Leaf> balance(const std::vector<Leaf>& t);
// Uniform base level, then every leaf below max_level whose gradient bound
// h sum_i |a_i| g(d_i) exceeds tol sum_i |a_i| is split, until none is; then balance.
std::vector<Leaf> refine_gaussians(int base_level, int max_level, int count, const double* centres,
                                   const double* sigma, const double* amps, double tol);
// Uniform base level, then every leaf below max_level with h max|f'| > tol max|f| is split,
// until none is; then balance.  f = -Laplace(u) for u = exp(-(r/R)^alpha), r the periodic
// distance to centre; the maxima come from a radial table with spacing R / (16 alpha),
// over the table entries covering the leaf's distance range.
std::vector<Leaf> refine_sharp_layer(int base_level, int max_level, const double* centre, double R, double alpha,
                                     double tol);
// Merge every complete family of 8 sibling leaves with parent level >= min_level, then balance.
std::vector<Leaf> coarsen(const std::vector<Leaf>& t, int min_level);

struct Csr {
  int64_t rows = 0, cols = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};
Csr transpose(const Csr& a);

// The continuous order-q (q = 1, 2) space on one octree.
struct Space {
  int q = 0;
  int m = 0;                        // (q+1)^3 nodes per element
  std::vector<Leaf> leaves;         // Morton order
  std::vector<uint64_t> keys;       // Morton keys of the anchors
  std::vector<int64_t> points;      // tick key x + T (y + T z) of each DoF, ascending
  Csr C;                            // (E m) x ndof: element node -> DoFs (constraints resolved)
  int64_t ndof() const { return static_cast<int64_t>(points.size()); }
  int64_t elements() const { return static_cast<int64_t>(leaves.size()); }
  int find(int64_t cx, int64_t cy, int64_t cz) const;  // leaf holding unit cell (wrapped)
};

// kref / mref: reference element stiffness / mass of the unit cube, m x m row-major
// (an element of width h has h kref and h^3 mref).
Space build_space(const std::vector<Leaf>& t, int q);
std::vector<double> element_diag_sum(const Space& s, const std::vector<double>& kref);  // diag(C^T A_e C)
std::vector<double> basis_integrals(const Space& s, const std::vector<double>& mref);   // C^T (h^3 mref 1)
std::vector<double> dense_operator(const Space& s, const std::vector<double>& kref);    // C^T A_e C, dense
// Row p of P: the coarse interpolant at fine DoF p (eq. 2.2), fine ndof x coarse ndof.
Csr prolongation(const Space& coarse, const Space& fine);
// Reference element matrices of the unit cube for order q (tensor products of the 1D ones).
void reference_element(int q, std::vector<double>* kref, std::vector<double>* mref);

}  // namespace oct
}  // namespace gmg
