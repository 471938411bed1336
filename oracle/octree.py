"""Periodic linear octree: refinement, 2:1 balance, coarsening (oracle, test infrastructure).

Paper: Section 2.3.1 builds the multigrid hierarchy on a Morton-ordered linear
octree: coarsening merges the 8 siblings of a family (which sit together in
Morton order), then the 2:1 balance is enforced again, and the recursion stops
when no further coarsening is possible; Section 2.2.1 defines the 2:1 balance
(adjacent leaves differ in depth by at most one) and balance refinement;
Section 3 (software parameters) drives the adaptivity of the multigrid runs by
the gradient of f.  The algorithms here are written from those statements.

Readings (the paper is silent on them):
  * "Adjacent" is taken as touching across a face, an edge or a corner, on the
    periodic unit cube (leaves wrap around).
  * Coarsening merges every family of 8 sibling leaves whose parent is not
    coarser than the coarsest multigrid level, all at once, then balances.
    Balancing only refines, so the result is nested in the finer tree.
  * Refinement of the adaptive workload: split leaf O while its level is below
    the maximum and  h_O sum_i |a_i| g(d_i) > tol sum_i |a_i|,  where d_i is the
    periodic distance from Gaussian centre c_i to the box O and
    g(d) = (d'/s_i^2) exp(-d'^2 / (2 s_i^2)) with d' = max(d, s_i): an upper
    bound of |grad| of the Gaussian a_i exp(-r^2 / (2 s_i^2)) over the box.

  * Refinement for the sharp-layer solution u = exp(-(r/R)^alpha) of the time-to-
    solution test case (Section 3; f = -Laplace(u) in closed form): split leaf O
    while its level is below the maximum and  h_O max|f'| > tol max|f|, the maxima
    taken over a radial table of |f'(r)| and |f(r)| at r_j = j dr,
    dr = R / (16 alpha), with the box's periodic distance range [d_min, d_max]
    from the centre covered by the table entries floor(d_min/dr) .. ceil(d_max/dr).
    The table spacing is a sixteenth of the layer width R / alpha, so the peak of
    |f'| near r = R is not missed between entries.

Representation: a leaf is (level, x, y, z) with its anchor in units of
2^-DMAX; its Morton key interleaves the anchor bits with x in the lowest bit.
A linear octree is a list of leaves sorted by Morton key.

Pins (tests/test_oracle_octree.py): the balanced tree is 2:1 across every
touching pair (brute force over all pairs), refines its input, and is minimal
(undoing any split that balancing made breaks the balance); refinement stops
exactly where the criterion says; coarsening nests and ends uniform.

Not a product path: only the tests, the smoke check and the CPU baseline use it.
"""
import math

import numpy as np

DMAX = 10
UNITS = 1 << DMAX


def size(level):
    return 1 << (DMAX - level)


def morton(x, y, z):
    """Interleaved bits of (x, y, z), x lowest."""
    k = 0
    for b in range(DMAX):
        k |= ((x >> b) & 1) << (3 * b)
        k |= ((y >> b) & 1) << (3 * b + 1)
        k |= ((z >> b) & 1) << (3 * b + 2)
    return k


def sort_leaves(leaves):
    return sorted(leaves, key=lambda o: morton(o[1], o[2], o[3]))


def uniform(level):
    s = size(level)
    r = range(0, UNITS, s)
    return sort_leaves([(level, x, y, z) for z in r for y in r for x in r])


def children(o):
    l, x, y, z = o
    s = size(l + 1)
    return [(l + 1, x + dx * s, y + dy * s, z + dz * s) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]


def parent(o):
    l, x, y, z = o
    s = size(l - 1)
    return (l - 1, x - x % s, y - y % s, z - z % s)


def is_linear_complete(leaves):
    """Sorted by Morton key, anchors aligned, Morton ranges contiguous and covering the cube."""
    pos = 0
    for l, x, y, z in leaves:
        if not (0 <= l <= DMAX):
            return False
        s = size(l)
        if x % s or y % s or z % s or not (0 <= x < UNITS and 0 <= y < UNITS and 0 <= z < UNITS):
            return False
        if morton(x, y, z) != pos:
            return False
        pos += s ** 3
    return pos == UNITS ** 3


class Locator:
    """Leaf containing a unit cell, by trying every level (a dict lookup each)."""

    def __init__(self, leaves):
        self.set = set(leaves)
        self.levels = sorted({o[0] for o in leaves})

    def find(self, x, y, z):
        x, y, z = x % UNITS, y % UNITS, z % UNITS
        for l in self.levels:
            s = size(l)
            o = (l, x - x % s, y - y % s, z - z % s)
            if o in self.set:
                return o
        raise KeyError("cell not covered")


DIRS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if (dx, dy, dz) != (0, 0, 0)]


def probe(o, d):
    """A unit cell just outside leaf o in direction d (inside o's extent along d_k = 0)."""
    l, x, y, z = o
    s = size(l)
    return tuple((a - 1) if dk < 0 else (a + s if dk > 0 else a) for a, dk in zip((x, y, z), d))


def violators(leaves):
    """Leaves that touch a leaf two or more levels finer (must be split)."""
    loc = Locator(leaves)
    bad = set()
    for o in leaves:
        for d in DIRS:
            nb = loc.find(*probe(o, d))
            if nb[0] < o[0] - 1:
                bad.add(nb)
    return bad


def balance(leaves):
    """Coarsest 2:1-balanced refinement of a complete linear octree."""
    cur = set(leaves)
    while True:
        bad = violators(list(cur))
        if not bad:
            return sort_leaves(cur)
        for o in bad:
            cur.remove(o)
            cur.update(children(o))


def periodic_box_distance(c, lo, h):
    """Distance from point c to the box [lo, lo + h]^3 on the unit torus."""
    d2 = 0.0
    for k in range(3):
        best = math.inf
        for m in (-1.0, 0.0, 1.0):
            ck = c[k] + m
            dk = max(0.0, lo[k] - ck, ck - (lo[k] + h))
            best = min(best, dk)
        d2 += best * best
    return math.sqrt(d2)


def gradient_indicator(o, centres, sigma, amps):
    """h_O sum_i |a_i| g(d_i) for leaf o (see the module docstring)."""
    l, x, y, z = o
    h = 1.0 / (1 << l)
    lo = (x / UNITS, y / UNITS, z / UNITS)
    tot = 0.0
    for c, s, a in zip(centres, sigma, amps):
        d = max(periodic_box_distance(c, lo, h), s)
        tot += abs(a) * (d / (s * s)) * math.exp(-d * d / (2.0 * s * s))
    return h * tot


def periodic_box_distance_range(c, lo, h):
    """(d_min, d_max): least and greatest periodic (nearest-image) distance from point c
    to the points of the box [lo, lo + h]^3 on the unit torus."""
    d2min = 0.0
    d2max = 0.0
    for k in range(3):
        best = math.inf
        for m in (-1.0, 0.0, 1.0):
            ck = c[k] + m
            best = min(best, max(0.0, lo[k] - ck, ck - (lo[k] + h)))
        # the nearest-image distance along one axis is a tent in x with its top at the
        # point opposite c; over [lo, lo + h] it is largest at an end or at that top
        def tent(x):
            d = abs(x - c[k]) % 1.0
            return min(d, 1.0 - d)
        far = max(tent(lo[k]), tent(lo[k] + h))
        opp = (c[k] + 0.5) % 1.0
        if lo[k] <= opp <= lo[k] + h or lo[k] <= opp + 1.0 <= lo[k] + h:
            far = 0.5
        d2min += best * best
        d2max += far * far
    return math.sqrt(d2min), math.sqrt(d2max)


def sharp_layer_profile(r, R, alpha):
    """(f(r), f'(r)) of f = -Laplace(u), u = exp(-s), s = (r/R)^alpha, written from
    u' = -e^-s s', s' = alpha s / r:  f = e^-s (alpha s / r^2) (alpha + 1 - alpha s)."""
    if r <= 0.0:
        return 0.0, 0.0
    s = math.exp(alpha * math.log(r / R))
    e = math.exp(-s)
    g = s / (r * r)
    w = alpha + 1.0 - alpha * s
    f = e * alpha * g * w
    # d/dr of e^-s alpha g w, with s' = alpha s / r, g' = (alpha - 2) g / r, w' = -alpha s'
    fp = alpha * e * (g / r) * (-alpha * s * w - alpha * alpha * s + w * (alpha - 2.0))
    return f, fp


def sharp_layer_table(R, alpha):
    """(dr, |f'(r_j)|, max |f|) on r_j = j dr up to the largest periodic distance."""
    dr = R / (16.0 * alpha)
    count = int(math.ceil(math.sqrt(3.0) / 2.0 / dr)) + 2
    fpabs = []
    fmax = 0.0
    for j in range(count):
        f, fp = sharp_layer_profile(j * dr, R, alpha)
        fpabs.append(abs(fp))
        fmax = max(fmax, abs(f))
    return dr, fpabs, fmax


def sharp_layer_indicator(o, centre, table):
    """h_O max |f'| over the table entries covering O's distance range from the centre."""
    dr, fpabs, _ = table
    l, x, y, z = o
    h = 1.0 / (1 << l)
    dmin, dmax = periodic_box_distance_range(centre, (x / UNITS, y / UNITS, z / UNITS), h)
    j0 = int(math.floor(dmin / dr))
    j1 = min(int(math.ceil(dmax / dr)), len(fpabs) - 1)
    return h * max(fpabs[j0:j1 + 1])


def refine_sharp_layer(base_level, max_level, centre, R, alpha, tol=1e-2):
    """Uniform base, split every leaf whose indicator exceeds tol max|f| (below max_level),
    until none does; then 2:1 balance."""
    table = sharp_layer_table(R, alpha)
    thresh = tol * table[2]
    todo = uniform(base_level)
    done = []
    while todo:
        nxt = []
        for o in todo:
            if o[0] < max_level and sharp_layer_indicator(o, centre, table) > thresh:
                nxt.extend(children(o))
            else:
                done.append(o)
        todo = nxt
    return balance(sort_leaves(done))


def refine_gaussians(base_level, max_level, centres, sigma, amps, tol=1e-2):
    """The adaptive tree: refine_by_indicator, then 2:1 balance."""
    return balance(refine_by_indicator(base_level, max_level, centres, sigma, amps, tol))


def refine_by_indicator(base_level, max_level, centres, sigma, amps, tol=1e-2):
    """Uniform base, split every leaf whose indicator exceeds tol sum|a| (below max_level),
    repeated until none does (not balanced)."""
    thresh = tol * float(np.sum(np.abs(amps)))
    todo = uniform(base_level)
    done = []
    while todo:
        nxt = []
        for o in todo:
            if o[0] < max_level and gradient_indicator(o, centres, sigma, amps) > thresh:
                nxt.extend(children(o))
            else:
                done.append(o)
        todo = nxt
    return sort_leaves(done)


def coarsen(leaves, min_level):
    """Merge every complete family of 8 sibling leaves with parent level >= min_level, then balance."""
    cur = set(leaves)
    parents = {}
    for o in leaves:
        if o[0] > min_level:
            parents.setdefault(parent(o), []).append(o)
    for p, kids in parents.items():
        if len(kids) == 8:
            cur.difference_update(kids)
            cur.add(p)
    return balance(sort_leaves(cur))


def hierarchy(leaves, min_level):
    """Trees from coarsest (uniform at min_level) to finest (the input)."""
    trees = [sort_leaves(leaves)]
    while any(o[0] != min_level for o in trees[-1]):
        trees.append(coarsen(trees[-1], min_level))
    return trees[::-1]
