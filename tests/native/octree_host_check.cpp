// Host octree meshing and setup arithmetic under AddressSanitizer and UBSan (CPU only).
// Builds adaptive octrees, balances, coarsens down to the uniform level-2 mesh, builds the
// Q1 / Q2 spaces and prolongations of every level, and checks invariants that any out-of-
// bounds or uninitialised access would most likely break.  Exit status 0 on success.
#include <cmath>
#include <cstdio>
#include <vector>

#include "gmg_octree_host.h"
#include "gmg_setup_math.h"

using namespace gmg;

static int fails = 0;
#define CHECK(c)                                                       \
  do {                                                                 \
    if (!(c)) {                                                        \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++fails;                                                         \
    }                                                                  \
  } while (0)

int main() {
  const double centres[6] = {0.3, 0.7, 0.1, 0.95, 0.05, 0.5};
  const double sigma[2] = {0.01, 0.02};
  const double amps[2] = {1.0, -0.5};
  for (int q : {1, 2}) {
    std::vector<oct::Leaf> t = oct::refine_gaussians(2, 6, 2, centres, sigma, amps, 1e-2);
    CHECK(oct::is_complete(t));
    CHECK(oct::is_balanced(t));
    std::vector<std::vector<oct::Leaf>> trees{t};
    while (true) {
      bool uniform = true;
      for (const auto& o : trees.back()) uniform = uniform && o.level == 2;
      if (uniform) break;
      trees.push_back(oct::coarsen(trees.back(), 2));
      CHECK(oct::is_complete(trees.back()) && oct::is_balanced(trees.back()));
    }
    std::vector<double> kref, mref;
    oct::reference_element(q, &kref, &mref);
    std::vector<oct::Space> sp;
    for (auto it = trees.rbegin(); it != trees.rend(); ++it) sp.push_back(oct::build_space(*it, q));
    for (size_t l = 0; l < sp.size(); ++l) {
      const oct::Space& s = sp[l];
      CHECK(s.C.rows == s.elements() * s.m && s.C.ptr.back() == static_cast<int64_t>(s.C.col.size()));
      for (int32_t c : s.C.col) CHECK(c >= 0 && c < s.ndof());
      std::vector<double> d = oct::element_diag_sum(s, kref);
      for (double v : d) CHECK(v > 0.0);
      std::vector<double> w = oct::basis_integrals(s, mref);
      double tot = 0.0;
      for (double v : w) tot += v;
      CHECK(std::fabs(tot - 1.0) < 1e-12);
      if (l > 0) {
        const oct::Csr P = oct::prolongation(sp[l - 1], s);
        for (int64_t i = 0; i < P.rows; ++i) {
          double rs = 0.0;
          for (int64_t j = P.ptr[i]; j < P.ptr[i + 1]; ++j) rs += P.val[j];
          CHECK(std::fabs(rs - 1.0) < 1e-13);
        }
        const oct::Csr R = oct::transpose(P);
        CHECK(R.rows == P.cols && R.col.size() == P.col.size());
      }
    }
    // the coarsest level is dense: A 1 = 0 and its pseudo-inverse exists
    const int64_t n0 = sp[0].ndof();
    std::vector<double> A = oct::dense_operator(sp[0], kref);
    double amax = 0.0, rmax = 0.0;
    for (int64_t i = 0; i < n0; ++i) {
      double r = 0.0;
      for (int64_t j = 0; j < n0; ++j) {
        r += A[i * n0 + j];
        amax = std::fmax(amax, std::fabs(A[i * n0 + j]));
      }
      rmax = std::fmax(rmax, std::fabs(r));
    }
    CHECK(rmax < 1e-12 * amax);
    std::vector<double> inv = dense_pseudo_inverse(A, static_cast<int>(n0));
    CHECK(inv.size() == static_cast<size_t>(n0 * n0));
    std::printf("q=%d: %zu levels, finest %lld leaves %lld DoFs\n", q, sp.size(),
                static_cast<long long>(sp.back().elements()), static_cast<long long>(sp.back().ndof()));
  }
  return fails == 0 ? 0 : 1;
}
