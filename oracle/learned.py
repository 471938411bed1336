"""Learned smoother: a 3-layer convolutional residual-to-correction map.

The paper states that its smoother choice is heuristic (Section 1, Limitations;
Section 2.3.3); the learned smoother is not in the paper and follows the
reading recorded for this build:

  net      Conv3d(1->16) -> ReLU -> Conv3d(16->16) -> ReLU -> Conv3d(16->1),
           3x3x3 kernels, circular padding on the DoF lattice, no bias
           (16*27 + 16*16*27 + 16*27 = 7776 weights);
  input    x = D^-1 r / s with s = RMS(D^-1 r); output  e~ = s N(x);
  BF16     weights, the input and both hidden activations are rounded to BF16
           (round to nearest even) where the GPU kernels round them;
           accumulation is exact here (FP64), FP32 on the GPU;
  backward g2 = bf16(1[a2 > 0] (W3^T * gy)), g1 = bf16(1[a1 > 0] (W2^T * g2)),
           weight gradients accumulated over every voxel;
  loss     energy:   ||e - e~||_A^2 / ||e||_A^2 with e = A^+ r;
           residual: ||r - A e~||_2^2 / ||r||_2^2, the squared contraction of
           the residual in the norm the per-cycle fallback measures.

Lattice arrays are (N, N, N) indexed [z, y, x]; hidden activations are
(N, N, N, C) channels-last.  Tap t = (dz+1)*9 + (dy+1)*3 + (dx+1); a
convolution is a cross-correlation: out(v) = sum_t W[.., t] in(v + off(t)).

Pins (tests/test_oracle_learned.py): central finite differences of the FP64
network and of both losses through the network; identity weights reduce the
learned correction to damped Jacobi; zero weights give a zero correction; the
losses vanish at the exact correction and equal 1 at the zero correction.
"""
import numpy as np

NC = 16
NTAP = 27
SIZES = (NC * NTAP, NC * NC * NTAP, NC * NTAP)


def offsets():
    """(dz, dy, dx) of tap t = (dz+1)*9 + (dy+1)*3 + (dx+1)."""
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def bf16(a):
    """Round to the nearest BF16 value, ties to even (via the FP32 bit pattern)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def split(w):
    """Flat weight vector -> W1 (16, 27), W2 (16 out, 16 in, 27), W3 (16, 27)."""
    w = np.asarray(w, dtype=np.float64)
    a, b, _ = SIZES
    return w[:a].reshape(NC, NTAP), w[a:a + b].reshape(NC, NC, NTAP), w[a + b:].reshape(NC, NTAP)


def join(W1, W2, W3):
    return np.concatenate([W1.ravel(), W2.ravel(), W3.ravel()])


def shift(a, off):
    """a(v + off) with periodic wrap, for a [z, y, x, ...] array."""
    dz, dy, dx = off
    return np.roll(a, shift=(-dz, -dy, -dx), axis=(0, 1, 2))


def forward(w, x, emulate_bf16=True):
    """Forward pass on the input lattice x (N, N, N); returns (y, cache)."""
    rnd = bf16 if emulate_bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    W1, W2, W3 = (rnd(W) for W in split(w))
    xin = rnd(x)
    offs = offsets()
    z1 = np.zeros(x.shape + (NC,))
    for t, o in enumerate(offs):
        z1 += shift(xin, o)[..., None] * W1[:, t]
    a1 = rnd(np.maximum(z1, 0.0))
    z2 = np.zeros_like(z1)
    for t, o in enumerate(offs):
        z2 += shift(a1, o) @ W2[:, :, t].T
    a2 = rnd(np.maximum(z2, 0.0))
    y = np.zeros(x.shape)
    for t, o in enumerate(offs):
        y += shift(a2, o) @ W3[:, t]
    return y, (xin, a1, a2, (W1, W2, W3), rnd)


def backward(cache, gy, want_gin=False):
    """Gradients of sum(gy * y) w.r.t. the flat weights (and the input)."""
    xin, a1, a2, (W1, W2, W3), rnd = cache
    offs = offsets()
    # layer 3: y(v) = sum_t a2(v + o_t) . W3[:, t]
    g2 = np.zeros(a2.shape)
    gW3 = np.zeros_like(W3)
    for t, o in enumerate(offs):
        g2 += shift(gy, tuple(-c for c in o))[..., None] * W3[:, t]
        gW3[:, t] = np.einsum("zyxc,zyx->c", shift(a2, o), gy)
    g2 = rnd(g2 * (a2 > 0))
    # layer 2: z2(v) = sum_t W2[:, :, t] a1(v + o_t)
    g1 = np.zeros(a1.shape)
    gW2 = np.zeros_like(W2)
    for t, o in enumerate(offs):
        g1 += shift(g2, tuple(-c for c in o)) @ W2[:, :, t]
        gW2[:, :, t] = np.einsum("zyxo,zyxi->oi", g2, shift(a1, o))
    g1 = rnd(g1 * (a1 > 0))
    # layer 1: z1(v) = sum_t W1[:, t] xin(v + o_t)
    gW1 = np.zeros_like(W1)
    gin = np.zeros(xin.shape) if want_gin else None
    for t, o in enumerate(offs):
        gW1[:, t] = np.einsum("zyxc,zyx->c", g1, shift(xin, o))
        if want_gin:
            gin += shift(g1, tuple(-c for c in o)) @ W1[:, t]
    return join(gW1, gW2, gW3), gin


def correction(w, r, dinv, emulate_bf16=True):
    """Learned correction e~ = s N(D^-1 r / s), s = RMS(D^-1 r), on the (N, N, N) lattice."""
    t = dinv * r
    s = np.sqrt(np.mean(t * t))
    if s == 0.0:
        return np.zeros_like(r), 0.0
    y, _ = forward(w, t / s, emulate_bf16)
    return s * y, s


def loss(A, e, e_tilde):
    """||e - e~||_A^2 / ||e||_A^2 (A a matrix acting on flat vectors)."""
    d = (e - e_tilde).ravel()
    return float(d @ (A @ d)) / float(e.ravel() @ (A @ e.ravel()))


def residual_loss(A, r, e_tilde):
    """||r - A e~||_2^2 / ||r||_2^2 (A a matrix acting on flat vectors)."""
    d = r.ravel() - A @ e_tilde.ravel()
    return float(d @ d) / float(r.ravel() @ r.ravel())


def loss_and_gradient(w, A, dinv, r, e=None, kind="energy", emulate_bf16=True):
    """Loss of one pair and its gradient with respect to the flat weights.

    e~ = s y with y = N(D^-1 r / s); s depends on r alone, so dL/dy = s dL/de~ with
      energy    dL/de~ = -2 A (e - e~) / ||e||_A^2
      residual  dL/de~ = -2 A (r - A e~) / ||r||_2^2
    and dL/dw is the network's backward pass applied to dL/dy.  r, e, dinv are
    (N, N, N) lattices; A acts on flat vectors."""
    t = dinv * r
    s = np.sqrt(np.mean(t * t))
    y, cache = forward(w, t / s, emulate_bf16)
    et = (s * y).ravel()
    if kind == "energy":
        ev = e.ravel()
        diff = ev - et
        Ae = A @ ev
        val = float(diff @ (A @ diff)) / float(ev @ Ae)
        g_et = -2.0 * (A @ diff) / float(ev @ Ae)
    elif kind == "residual":
        d = r.ravel() - A @ et
        rr = float(r.ravel() @ r.ravel())
        val = float(d @ d) / rr
        g_et = -2.0 * (A.T @ d) / rr
    else:
        raise ValueError(kind)
    g, _ = backward(cache, (s * g_et).reshape(y.shape))
    return val, g


def jacobi_weights(omega):
    """Weights with N(x) = omega (ReLU(x) - ReLU(-x)) = omega x through two channels, centre taps only."""
    W1 = np.zeros((NC, NTAP))
    W2 = np.zeros((NC, NC, NTAP))
    W3 = np.zeros((NC, NTAP))
    c = 13  # (0, 0, 0)
    W1[0, c], W1[1, c] = 1.0, -1.0
    W2[0, 0, c], W2[1, 1, c] = 1.0, 1.0
    W3[0, c], W3[1, c] = omega, -omega
    return join(W1, W2, W3)


def init_weights(seed, scale=None):
    """He-style initialization, seeded: N(0, 2/fan_in) per layer (layer 3 scaled by 0.1)."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((NC, NTAP)) * np.sqrt(2.0 / NTAP)
    W2 = rng.standard_normal((NC, NC, NTAP)) * np.sqrt(2.0 / (NC * NTAP))
    W3 = rng.standard_normal((NC, NTAP)) * np.sqrt(2.0 / (NC * NTAP)) * 0.1
    return join(W1, W2, W3)
