// Periodic linear octree and continuous Q_q space with hanging nodes (host).
//
// Octree (Section 2.3.1): leaves in Morton order; a family of 8 siblings is a
// contiguous run, so splitting a leaf in place (children in Morton order) or
// merging a family keeps the order.  2:1 balance (Section 2.2.1) is enforced
// across faces, edges and corners of the periodic cube by repeated splitting of
// every leaf that touches a leaf two or more levels finer; only leaves that any
// balanced refinement must split are split, so the fixed point is the coarsest
// balanced refinement.
//
// Space (Section 2.3, hanging nodes Section 4): node positions live on a lattice
// of 2^(kMaxLevel+1) ticks per unit length.  A node position is a degree of
// freedom iff it is a node of the coarsest leaf whose closed box contains it;
// otherwise it hangs and takes that leaf's Q_q interpolant, resolved
// recursively.  DoFs are numbered by ascending tick key x + T (y + T z).
#include "gmg_octree_host.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <stdexcept>
#include <thread>
#include <unordered_map>

#include "gmg_setup_math.h"

namespace gmg {
namespace oct {

namespace {

inline uint64_t spread3(uint32_t v) {
  uint64_t r = 0;
  for (int b = 0; b < kMaxLevel; ++b) r |= static_cast<uint64_t>((v >> b) & 1u) << (3 * b);
  return r;
}

inline int32_t wrap(int64_t v, int64_t m) { return static_cast<int32_t>(((v % m) + m) % m); }

inline uint64_t key_of(const Leaf& o) { return morton_key(o.x, o.y, o.z); }

// Locate the leaf holding a unit cell in a Morton-sorted complete octree.
int locate(const std::vector<uint64_t>& keys, int64_t cx, int64_t cy, int64_t cz) {
  const uint64_t k = morton_key(wrap(cx, kUnits), wrap(cy, kUnits), wrap(cz, kUnits));
  const auto it = std::upper_bound(keys.begin(), keys.end(), k);
  return static_cast<int>(it - keys.begin()) - 1;
}

std::vector<uint64_t> keys_of(const std::vector<Leaf>& t) {
  std::vector<uint64_t> k(t.size());
  for (size_t i = 0; i < t.size(); ++i) k[i] = key_of(t[i]);
  return k;
}

// f(i) for i in [0, n) on up to 16 host threads, in contiguous chunks (the calls
// must be independent); serial below min_n items.
template <typename F>
void parallel_for(int64_t n, const F& f, int64_t min_n = int64_t{1} << 16) {
  unsigned nt = std::thread::hardware_concurrency();
  nt = std::max(1u, std::min(nt, 16u));
  if (n < min_n) nt = 1;
  if (nt == 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  const int64_t chunk = (n + nt - 1) / nt;
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t) {
    const int64_t b = t * chunk, e = std::min<int64_t>(n, b + chunk);
    if (b < e) th.emplace_back([&f, b, e] {
      for (int64_t i = b; i < e; ++i) f(i);
    });
  }
  for (auto& x : th) x.join();
}

void push_children(const Leaf& o, std::vector<Leaf>* out) {
  const int32_t s = leaf_size(o.level + 1);
  for (int c = 0; c < 8; ++c)  // child c = dx + 2 dy + 4 dz is also its Morton rank
    out->push_back({o.x + (c & 1) * s, o.y + ((c >> 1) & 1) * s, o.z + ((c >> 2) & 1) * s, o.level + 1});
}

// Mark every leaf that touches leaf i from outside and is >= 2 levels coarser.
void mark_coarse_neighbours(const std::vector<Leaf>& t, const std::vector<uint64_t>& keys, size_t i,
                            std::vector<char>* split) {
  const Leaf& o = t[i];
  const int32_t s = leaf_size(o.level);
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        if (!dx && !dy && !dz) continue;
        // one unit cell just outside o in this direction; any leaf at least twice
        // o's width that touches o there holds it (aligned intervals nest)
        const int64_t px = dx < 0 ? o.x - 1 : (dx > 0 ? o.x + s : o.x);
        const int64_t py = dy < 0 ? o.y - 1 : (dy > 0 ? o.y + s : o.y);
        const int64_t pz = dz < 0 ? o.z - 1 : (dz > 0 ? o.z + s : o.z);
        const int j = locate(keys, px, py, pz);
        if (t[j].level < o.level - 1) (*split)[j] = 1;
      }
}

double box_distance(const double* c, const double lo[3], double h) {
  double d2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    double best = INFINITY;
    for (int m = -1; m <= 1; ++m) {
      const double ck = c[k] + m;
      best = std::min(best, std::max({0.0, lo[k] - ck, ck - (lo[k] + h)}));
    }
    d2 += best * best;
  }
  return std::sqrt(d2);
}

double indicator(const Leaf& o, int count, const double* centres, const double* sigma, const double* amps) {
  const double h = 1.0 / static_cast<double>(1 << o.level);
  const double lo[3] = {o.x / static_cast<double>(kUnits), o.y / static_cast<double>(kUnits),
                        o.z / static_cast<double>(kUnits)};
  double tot = 0.0;
  for (int i = 0; i < count; ++i) {
    const double s = sigma[i];
    const double d = std::max(box_distance(centres + 3 * i, lo, h), s);
    tot += std::fabs(amps[i]) * (d / (s * s)) * std::exp(-d * d / (2.0 * s * s));
  }
  return h * tot;
}

std::vector<Leaf> uniform(int level) {
  std::vector<Leaf> t;
  const int32_t s = leaf_size(level);
  const int64_t n = static_cast<int64_t>(1) << (3 * level);
  t.reserve(n);
  for (int64_t i = 0; i < n; ++i) {
    uint32_t x, y, z;
    morton_decode(static_cast<uint64_t>(i) * s * s * s, &x, &y, &z);
    t.push_back({static_cast<int32_t>(x), static_cast<int32_t>(y), static_cast<int32_t>(z), level});
  }
  return t;
}

// 1D Lagrange values of the order-q nodes {0, 1/2, 1} (q = 2) or {0, 1} (q = 1) at t.
void basis_1d(int q, double t, double* out) {
  if (q == 1) {
    out[0] = 1.0 - t;
    out[1] = t;
  } else {
    out[0] = 2.0 * (t - 0.5) * (t - 1.0);
    out[1] = -4.0 * t * (t - 1.0);
    out[2] = 2.0 * t * (t - 0.5);
  }
}

}  // namespace

uint64_t morton_key(uint32_t x, uint32_t y, uint32_t z) { return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2); }

void morton_decode(uint64_t key, uint32_t* x, uint32_t* y, uint32_t* z) {
  *x = *y = *z = 0;
  for (int b = 0; b < kMaxLevel; ++b) {
    *x |= static_cast<uint32_t>((key >> (3 * b)) & 1u) << b;
    *y |= static_cast<uint32_t>((key >> (3 * b + 1)) & 1u) << b;
    *z |= static_cast<uint32_t>((key >> (3 * b + 2)) & 1u) << b;
  }
}

bool is_complete(const std::vector<Leaf>& t) {
  uint64_t pos = 0;
  for (const Leaf& o : t) {
    if (o.level < 0 || o.level > kMaxLevel) return false;
    const int32_t s = leaf_size(o.level);
    if (o.x < 0 || o.y < 0 || o.z < 0 || o.x >= kUnits || o.y >= kUnits || o.z >= kUnits) return false;
    if (o.x % s || o.y % s || o.z % s) return false;
    if (key_of(o) != pos) return false;
    pos += static_cast<uint64_t>(s) * s * s;
  }
  return pos == static_cast<uint64_t>(kUnits) * kUnits * kUnits;
}

namespace {

// Leaves that some leaf touches from two or more levels finer; the marks of each
// thread's range of leaves go to a vector of its own and are OR-ed together.
std::vector<char> coarse_neighbour_marks(const std::vector<Leaf>& t) {
  const std::vector<uint64_t> keys = keys_of(t);
  const int64_t n = static_cast<int64_t>(t.size());
  unsigned nt = std::max(1u, std::min(std::thread::hardware_concurrency(), 16u));
  if (n < (int64_t{1} << 16)) nt = 1;
  std::vector<std::vector<char>> marks(nt, std::vector<char>(t.size(), 0));
  const int64_t chunk = (n + nt - 1) / nt;
  parallel_for(
      nt,
      [&](int64_t k) {
        const int64_t b = k * chunk, e = std::min<int64_t>(n, b + chunk);
        for (int64_t i = b; i < e; ++i) mark_coarse_neighbours(t, keys, static_cast<size_t>(i), &marks[k]);
      },
      2);
  for (unsigned k = 1; k < nt; ++k)
    for (int64_t i = 0; i < n; ++i) marks[0][i] |= marks[k][i];
  return std::move(marks[0]);
}

}  // namespace

bool is_balanced(const std::vector<Leaf>& t) {
  const std::vector<char> split = coarse_neighbour_marks(t);
  return std::find(split.begin(), split.end(), 1) == split.end();
}

std::vector<Leaf> balance(const std::vector<Leaf>& t0) {
  std::vector<Leaf> t = t0;
  while (true) {
    const std::vector<char> split = coarse_neighbour_marks(t);
    if (std::find(split.begin(), split.end(), 1) == split.end()) return t;
    std::vector<Leaf> next;
    next.reserve(t.size() + 7 * std::count(split.begin(), split.end(), 1));
    for (size_t i = 0; i < t.size(); ++i) {
      if (split[i]) push_children(t[i], &next);
      else next.push_back(t[i]);
    }
    t.swap(next);
  }
}

std::vector<Leaf> refine_gaussians(int base_level, int max_level, int count, const double* centres,
                                   const double* sigma, const double* amps, double tol) {
  double asum = 0.0;
  for (int i = 0; i < count; ++i) asum += std::fabs(amps[i]);
  const double thresh = tol * asum;
  std::vector<Leaf> t = uniform(base_level);
  while (true) {
    std::vector<Leaf> next;
    bool changed = false;
    for (const Leaf& o : t) {
      if (o.level < max_level && indicator(o, count, centres, sigma, amps) > thresh) {
        push_children(o, &next);
        changed = true;
      } else {
        next.push_back(o);
      }
    }
    t.swap(next);
    if (!changed) break;
  }
  return balance(t);
}

namespace {

// Least and greatest nearest-image distance from c to the box [lo, lo + h]^3.
void box_distance_range(const double* c, const double lo[3], double h, double* dmin, double* dmax) {
  double d2min = 0.0, d2max = 0.0;
  for (int k = 0; k < 3; ++k) {
    double best = INFINITY;
    for (int m = -1; m <= 1; ++m) {
      const double ck = c[k] + m;
      best = std::min(best, std::max({0.0, lo[k] - ck, ck - (lo[k] + h)}));
    }
    // the one-axis nearest-image distance is a tent with its top opposite c: over
    // [lo, lo + h] it is largest at an end or at that top
    auto tent = [&](double x) {
      const double d = std::fmod(std::fabs(x - c[k]), 1.0);
      return std::min(d, 1.0 - d);
    };
    double far = std::max(tent(lo[k]), tent(lo[k] + h));
    const double opp = std::fmod(c[k] + 0.5, 1.0);
    if ((lo[k] <= opp && opp <= lo[k] + h) || (lo[k] <= opp + 1.0 && opp + 1.0 <= lo[k] + h)) far = 0.5;
    d2min += best * best;
    d2max += far * far;
  }
  *dmin = std::sqrt(d2min);
  *dmax = std::sqrt(d2max);
}

// f = -Laplace(u) of u = exp(-s), s = (r/R)^alpha, and f' (radial):
// f = e^-s (alpha s / r^2) (alpha + 1 - alpha s).
void sharp_layer_profile(double r, double R, double alpha, double* f, double* fp) {
  if (r <= 0.0) {
    *f = 0.0;
    *fp = 0.0;
    return;
  }
  const double s = std::exp(alpha * std::log(r / R));
  const double e = std::exp(-s);
  const double g = s / (r * r);
  const double w = alpha + 1.0 - alpha * s;
  *f = e * alpha * g * w;
  // with s' = alpha s / r, g' = (alpha - 2) g / r, w' = -alpha s'
  *fp = alpha * e * (g / r) * (-alpha * s * w - alpha * alpha * s + w * (alpha - 2.0));
}

}  // namespace

std::vector<Leaf> refine_sharp_layer(int base_level, int max_level, const double* centre, double R, double alpha,
                                     double tol) {
  // |f'| on r_j = j dr, dr = R / (16 alpha) (a sixteenth of the layer width), and max |f|
  const double dr = R / (16.0 * alpha);
  const int count = static_cast<int>(std::ceil(std::sqrt(3.0) / 2.0 / dr)) + 2;
  std::vector<double> fpabs(count);
  double fmax = 0.0;
  for (int j = 0; j < count; ++j) {
    double f, fp;
    sharp_layer_profile(j * dr, R, alpha, &f, &fp);
    fpabs[j] = std::fabs(fp);
    fmax = std::max(fmax, std::fabs(f));
  }
  const double thresh = tol * fmax;
  auto indicator = [&](const Leaf& o) {
    const double h = 1.0 / static_cast<double>(1 << o.level);
    const double lo[3] = {o.x / static_cast<double>(kUnits), o.y / static_cast<double>(kUnits),
                          o.z / static_cast<double>(kUnits)};
    double dmin, dmax;
    box_distance_range(centre, lo, h, &dmin, &dmax);
    const int j0 = static_cast<int>(std::floor(dmin / dr));
    const int j1 = std::min(static_cast<int>(std::ceil(dmax / dr)), count - 1);
    double m = 0.0;
    for (int j = j0; j <= j1; ++j) m = std::max(m, fpabs[j]);
    return h * m;
  };
  std::vector<Leaf> t = uniform(base_level);
  while (true) {
    std::vector<Leaf> next;
    bool changed = false;
    for (const Leaf& o : t) {
      if (o.level < max_level && indicator(o) > thresh) {
        push_children(o, &next);
        changed = true;
      } else {
        next.push_back(o);
      }
    }
    t.swap(next);
    if (!changed) break;
  }
  return balance(t);
}

std::vector<Leaf> coarsen(const std::vector<Leaf>& t, int min_level) {
  std::vector<Leaf> out;
  out.reserve(t.size());
  size_t i = 0;
  while (i < t.size()) {
    const Leaf& o = t[i];
    if (o.level > min_level && i + 8 <= t.size()) {
      const int32_t ps = leaf_size(o.level - 1);
      bool family = o.x % ps == 0 && o.y % ps == 0 && o.z % ps == 0;
      for (int k = 1; family && k < 8; ++k) family = t[i + k].level == o.level;
      if (family) {  // first child and 8 leaves of its level: the whole Morton range of the parent
        out.push_back({o.x, o.y, o.z, o.level - 1});
        i += 8;
        continue;
      }
    }
    out.push_back(o);
    ++i;
  }
  return balance(out);
}

Csr transpose(const Csr& a) {
  Csr t;
  t.rows = a.cols;
  t.cols = a.rows;
  t.ptr.assign(t.rows + 1, 0);
  for (int32_t c : a.col) ++t.ptr[c + 1];
  for (int64_t r = 0; r < t.rows; ++r) t.ptr[r + 1] += t.ptr[r];
  t.col.resize(a.col.size());
  t.val.resize(a.val.size());
  std::vector<int64_t> fill(t.ptr.begin(), t.ptr.end() - 1);
  for (int64_t r = 0; r < a.rows; ++r)
    for (int64_t j = a.ptr[r]; j < a.ptr[r + 1]; ++j) {
      const int64_t d = fill[a.col[j]]++;
      t.col[d] = static_cast<int32_t>(r);
      t.val[d] = a.val[j];
    }
  return t;
}

int Space::find(int64_t cx, int64_t cy, int64_t cz) const { return locate(keys, cx, cy, cz); }

void reference_element(int q, std::vector<double>* kref, std::vector<double>* mref) {
  std::vector<double> k1, m1;
  reference_matrices(q, &k1, &m1);
  const int p = q + 1, m = p * p * p;
  kref->assign(static_cast<size_t>(m) * m, 0.0);
  mref->assign(static_cast<size_t>(m) * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      const int ia = i % p, ib = (i / p) % p, ic = i / (p * p);
      const int ja = j % p, jb = (j / p) % p, jc = j / (p * p);
      const double K[3] = {k1[ia * p + ja], k1[ib * p + jb], k1[ic * p + jc]};
      const double M[3] = {m1[ia * p + ja], m1[ib * p + jb], m1[ic * p + jc]};
      (*kref)[static_cast<size_t>(i) * m + j] = K[0] * M[1] * M[2] + M[0] * K[1] * M[2] + M[0] * M[1] * K[2];
      (*mref)[static_cast<size_t>(i) * m + j] = M[0] * M[1] * M[2];
    }
}

namespace {

// Node positions are identified by their rank in the sorted list of distinct element-node
// positions; each is either a DoF or hangs on a source leaf.
struct Builder {
  const Space& s;
  int p;                                      // nodes per direction (q + 1)
  std::vector<int64_t> elem_pos;              // (E m) tick keys
  std::vector<int64_t> uniq;                  // distinct positions, ascending
  std::vector<int32_t> rank_of;               // elem_pos index -> rank in uniq
  std::vector<int64_t> dof_of;                // rank -> DoF, or -1 where the position hangs
  std::vector<int32_t> src_of;                // rank -> leaf whose interpolant a hanging position takes
  std::vector<std::vector<std::pair<int64_t, double>>> memo;  // rank -> resolved weights (hanging)
  std::vector<char> done;

  static int64_t tkey(int64_t x, int64_t y, int64_t z) { return x + kTicks * (y + kTicks * z); }

  void local_ticks(const Leaf& o, int64_t key, int64_t t[3]) const {
    const int64_t pc[3] = {key % kTicks, (key / kTicks) % kTicks, key / (kTicks * kTicks)};
    const int64_t an[3] = {2 * static_cast<int64_t>(o.x), 2 * static_cast<int64_t>(o.y),
                           2 * static_cast<int64_t>(o.z)};
    for (int k = 0; k < 3; ++k) t[k] = wrap(pc[k] - an[k], kTicks);
  }

  // phi_a at the position (tick key) inside leaf o, a = ia + p (ib + p ic)
  void basis_at(const Leaf& o, int64_t key, std::vector<double>* phi) const {
    int64_t t[3];
    local_ticks(o, key, t);
    const double w = 2.0 * leaf_size(o.level);
    double b[3][3];
    for (int k = 0; k < 3; ++k) basis_1d(s.q, static_cast<double>(t[k]) / w, b[k]);
    phi->assign(static_cast<size_t>(p) * p * p, 0.0);
    for (int c = 0; c < p; ++c)
      for (int bb = 0; bb < p; ++bb)
        for (int a = 0; a < p; ++a) (*phi)[a + p * (bb + p * c)] = b[0][a] * b[1][bb] * b[2][c];
  }

  bool is_node(const Leaf& o, int64_t key) const {
    int64_t t[3];
    local_ticks(o, key, t);
    const int64_t step = 2 * static_cast<int64_t>(leaf_size(o.level)) / s.q;  // node spacing in ticks
    for (int k = 0; k < 3; ++k)
      if (t[k] % step != 0 || t[k] > 2 * static_cast<int64_t>(leaf_size(o.level))) return false;
    return true;
  }

  int coarsest_containing(int64_t key) const {
    const int64_t px = key % kTicks, py = (key / kTicks) % kTicks, pz = key / (kTicks * kTicks);
    int best = -1;
    for (int dz = -1; dz <= 0; ++dz)
      for (int dy = -1; dy <= 0; ++dy)
        for (int dx = -1; dx <= 0; ++dx) {
          const int j = s.find(wrap(px + dx, kTicks) >> 1, wrap(py + dy, kTicks) >> 1, wrap(pz + dz, kTicks) >> 1);
          if (best < 0 || s.leaves[j].level < s.leaves[best].level ||
              (s.leaves[j].level == s.leaves[best].level && j < best))
            best = j;
        }
    return best;
  }

  // weights of the hanging position of rank u on the DoFs, in ascending DoF order: the
  // source leaf's interpolant, node by node (a ascending), each node resolved in turn
  const std::vector<std::pair<int64_t, double>>& expand(int32_t u) {
    if (done[u]) return memo[u];
    const int e = src_of[u];
    std::vector<double> phi;
    basis_at(s.leaves[e], uniq[u], &phi);
    const int m = p * p * p;
    std::map<int64_t, double> out;
    for (int a = 0; a < m; ++a) {
      if (phi[a] == 0.0) continue;
      const int32_t v = rank_of[static_cast<size_t>(e) * m + a];
      if (dof_of[v] >= 0) {
        out[dof_of[v]] += phi[a] * 1.0;
      } else {
        const auto& sub = expand(v);
        for (const auto& kv : sub) out[kv.first] += phi[a] * kv.second;
      }
    }
    std::vector<std::pair<int64_t, double>> w;
    for (const auto& kv : out)
      if (kv.second != 0.0) w.push_back(kv);
    memo[u] = std::move(w);
    done[u] = 1;
    return memo[u];
  }
};

}  // namespace

Space build_space(const std::vector<Leaf>& t, int q) {
  if (q != 1 && q != 2) throw std::invalid_argument("octree spaces are built for q = 1, 2");
  Space s;
  s.q = q;
  const int p = q + 1;
  s.m = p * p * p;
  s.leaves = t;
  s.keys = keys_of(t);
  Builder B{s, p, {}, {}, {}, {}, {}, {}, {}};
  const int64_t E = s.elements();
  const int m = s.m;
  B.elem_pos.resize(static_cast<size_t>(E) * m);
  parallel_for(E, [&](int64_t e) {
    const Leaf& o = t[e];
    const int64_t step = 2 * static_cast<int64_t>(leaf_size(o.level)) / q;
    for (int c = 0; c < p; ++c)
      for (int b = 0; b < p; ++b)
        for (int a = 0; a < p; ++a)
          B.elem_pos[e * m + a + p * (b + p * c)] =
              Builder::tkey(wrap(2 * static_cast<int64_t>(o.x) + a * step, kTicks),
                            wrap(2 * static_cast<int64_t>(o.y) + b * step, kTicks),
                            wrap(2 * static_cast<int64_t>(o.z) + c * step, kTicks));
  });
  B.uniq = B.elem_pos;
  std::sort(B.uniq.begin(), B.uniq.end());
  B.uniq.erase(std::unique(B.uniq.begin(), B.uniq.end()), B.uniq.end());
  const int64_t U = static_cast<int64_t>(B.uniq.size());
  if (U > INT32_MAX) throw std::length_error("too many node positions");
  // DoF or hanging, per position (independent); DoFs numbered in ascending position order
  std::vector<char> is_dof(U);
  B.src_of.assign(U, -1);
  parallel_for(U, [&](int64_t u) {
    const int e = B.coarsest_containing(B.uniq[u]);
    is_dof[u] = B.is_node(t[e], B.uniq[u]);
    if (!is_dof[u]) B.src_of[u] = e;
  });
  B.dof_of.assign(U, -1);
  for (int64_t u = 0; u < U; ++u)
    if (is_dof[u]) {
      B.dof_of[u] = static_cast<int64_t>(s.points.size());
      s.points.push_back(B.uniq[u]);
    }
  B.rank_of.resize(B.elem_pos.size());
  parallel_for(static_cast<int64_t>(B.elem_pos.size()), [&](int64_t r) {
    B.rank_of[r] = static_cast<int32_t>(std::lower_bound(B.uniq.begin(), B.uniq.end(), B.elem_pos[r]) - B.uniq.begin());
  });
  // resolve every hanging position once (recursively, memoised)
  B.memo.resize(U);
  B.done.assign(U, 0);
  for (int64_t u = 0; u < U; ++u)
    if (!is_dof[u]) B.expand(static_cast<int32_t>(u));
  // C: one row per element node, its position's weights
  s.C.rows = E * m;
  s.C.cols = s.ndof();
  s.C.ptr.assign(s.C.rows + 1, 0);
  for (int64_t r = 0; r < s.C.rows; ++r) {
    const int32_t u = B.rank_of[r];
    s.C.ptr[r + 1] = s.C.ptr[r] + (is_dof[u] ? 1 : static_cast<int64_t>(B.memo[u].size()));
  }
  s.C.col.resize(s.C.ptr[s.C.rows]);
  s.C.val.resize(s.C.ptr[s.C.rows]);
  parallel_for(s.C.rows, [&](int64_t r) {
    const int32_t u = B.rank_of[r];
    int64_t k = s.C.ptr[r];
    if (is_dof[u]) {
      s.C.col[k] = static_cast<int32_t>(B.dof_of[u]);
      s.C.val[k] = 1.0;
      return;
    }
    for (const auto& kv : B.memo[u]) {
      s.C.col[k] = static_cast<int32_t>(kv.first);
      s.C.val[k] = kv.second;
      ++k;
    }
  });
  return s;
}

std::vector<double> element_diag_sum(const Space& s, const std::vector<double>& kref) {
  std::vector<double> d(s.ndof(), 0.0);
  const int m = s.m;
  for (int64_t e = 0; e < s.elements(); ++e) {
    const double h = 1.0 / static_cast<double>(1 << s.leaves[e].level);
    for (int a = 0; a < m; ++a)
      for (int b = 0; b < m; ++b) {
        const double kab = h * kref[static_cast<size_t>(a) * m + b];
        const int64_t ra = e * m + a, rb = e * m + b;
        for (int64_t i = s.C.ptr[ra]; i < s.C.ptr[ra + 1]; ++i)
          for (int64_t j = s.C.ptr[rb]; j < s.C.ptr[rb + 1]; ++j)
            if (s.C.col[i] == s.C.col[j]) d[s.C.col[i]] += s.C.val[i] * kab * s.C.val[j];
      }
  }
  return d;
}

std::vector<double> basis_integrals(const Space& s, const std::vector<double>& mref) {
  std::vector<double> w(s.ndof(), 0.0);
  const int m = s.m;
  std::vector<double> rowsum(m, 0.0);
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b) rowsum[a] += mref[static_cast<size_t>(a) * m + b];
  for (int64_t e = 0; e < s.elements(); ++e) {
    const double h = 1.0 / static_cast<double>(1 << s.leaves[e].level);
    for (int a = 0; a < m; ++a) {
      const int64_t r = e * m + a;
      for (int64_t i = s.C.ptr[r]; i < s.C.ptr[r + 1]; ++i) w[s.C.col[i]] += s.C.val[i] * h * h * h * rowsum[a];
    }
  }
  return w;
}

std::vector<double> dense_operator(const Space& s, const std::vector<double>& kref) {
  const int64_t n = s.ndof();
  std::vector<double> A(static_cast<size_t>(n) * n, 0.0);
  const int m = s.m;
  for (int64_t e = 0; e < s.elements(); ++e) {
    const double h = 1.0 / static_cast<double>(1 << s.leaves[e].level);
    for (int a = 0; a < m; ++a)
      for (int b = 0; b < m; ++b) {
        const double kab = h * kref[static_cast<size_t>(a) * m + b];
        const int64_t ra = e * m + a, rb = e * m + b;
        for (int64_t i = s.C.ptr[ra]; i < s.C.ptr[ra + 1]; ++i)
          for (int64_t j = s.C.ptr[rb]; j < s.C.ptr[rb + 1]; ++j)
            A[static_cast<size_t>(s.C.col[i]) * n + s.C.col[j]] += s.C.val[i] * kab * s.C.val[j];
      }
  }
  return A;
}

Csr prolongation(const Space& coarse, const Space& fine) {
  Csr P;
  P.rows = fine.ndof();
  P.cols = coarse.ndof();
  P.ptr.assign(P.rows + 1, 0);
  const int p = coarse.q + 1, m = coarse.m;
  for (int64_t i = 0; i < P.rows; ++i) {
    const int64_t key = fine.points[i];
    const int64_t px = key % kTicks, py = (key / kTicks) % kTicks, pz = key / (kTicks * kTicks);
    const int e = coarse.find(px >> 1, py >> 1, pz >> 1);
    const Leaf& o = coarse.leaves[e];
    const int64_t an[3] = {2 * static_cast<int64_t>(o.x), 2 * static_cast<int64_t>(o.y),
                           2 * static_cast<int64_t>(o.z)};
    const int64_t pc[3] = {px, py, pz};
    const double w = 2.0 * leaf_size(o.level);
    double b[3][3];
    for (int k = 0; k < 3; ++k) basis_1d(coarse.q, static_cast<double>(wrap(pc[k] - an[k], kTicks)) / w, b[k]);
    std::map<int32_t, double> row;
    for (int c = 0; c < p; ++c)
      for (int bb = 0; bb < p; ++bb)
        for (int a = 0; a < p; ++a) {
          const double phi = b[0][a] * b[1][bb] * b[2][c];
          if (phi == 0.0) continue;
          const int64_t r = static_cast<int64_t>(e) * m + a + p * (bb + p * c);
          for (int64_t j = coarse.C.ptr[r]; j < coarse.C.ptr[r + 1]; ++j) row[coarse.C.col[j]] += phi * coarse.C.val[j];
        }
    for (const auto& kv : row) {
      if (kv.second == 0.0) continue;
      P.col.push_back(kv.first);
      P.val.push_back(kv.second);
    }
    P.ptr[i + 1] = static_cast<int64_t>(P.col.size());
  }
  return P;
}

}  // namespace oct
}  // namespace gmg
