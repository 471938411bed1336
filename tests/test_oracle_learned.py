"""Pins of the oracle's learned smoother (a reading: the paper has no learned smoother)."""
import numpy as np
import pytest

from oracle import learned, operator as op


def _rand_weights(seed, scale=0.3):
    return np.random.default_rng(seed).standard_normal(sum(learned.SIZES)) * scale


@pytest.mark.parametrize("seed", [0, 1])
def test_weight_gradient_matches_central_differences(seed):
    N = 5
    rng = np.random.default_rng(100 + seed)
    x = rng.standard_normal((N, N, N))
    gy = rng.standard_normal((N, N, N))
    w = _rand_weights(seed)
    y, cache = learned.forward(w, x, emulate_bf16=False)
    g, gin = learned.backward(cache, gy, want_gin=True)
    f = lambda ww: float(np.sum(gy * learned.forward(ww, x, emulate_bf16=False)[0]))
    h = 1e-6
    idx = rng.choice(len(w), 40, replace=False)
    for i in idx:
        e = np.zeros_like(w)
        e[i] = h
        fd = (f(w + e) - f(w - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])
    fx = lambda xx: float(np.sum(gy * learned.forward(w, xx, emulate_bf16=False)[0]))
    for _ in range(10):
        j = tuple(rng.integers(0, N, 3))
        e = np.zeros_like(x)
        e[j] = h
        fd = (fx(x + e) - fx(x - e)) / (2 * h)
        assert abs(fd - gin[j]) <= 1e-6 * max(1.0, abs(fd))


def test_identity_weights_give_damped_jacobi():
    q, n = 2, 4
    A = op.assemble(q, n)
    N = q * n
    dinv = (1.0 / A.diagonal()).reshape(N, N, N)
    r = np.random.default_rng(3).standard_normal((N, N, N))
    omega = 0.7
    w = learned.jacobi_weights(omega)
    e_exact, _ = learned.correction(w, r, dinv, emulate_bf16=False)
    assert np.max(np.abs(e_exact - omega * dinv * r)) < 1e-13 * np.max(np.abs(dinv * r))
    # with BF16 rounding of the input (omega = 0.7 is not a BF16 value: rounded too)
    e_bf, s = learned.correction(w, r, dinv, emulate_bf16=True)
    wb = learned.bf16(omega)
    ref = s * wb * learned.bf16(dinv * r / s)
    assert np.max(np.abs(e_bf - ref)) < 1e-13 * np.max(np.abs(ref))
    assert np.max(np.abs(e_bf - omega * dinv * r)) <= 2 ** -7 * np.max(np.abs(dinv * r))


def test_zero_weights_zero_correction_and_loss_bounds():
    N = 4
    r = np.random.default_rng(0).standard_normal((N, N, N))
    e, s = learned.correction(np.zeros(sum(learned.SIZES)), r, np.ones_like(r))
    assert s > 0 and np.all(e == 0.0)
    A = op.assemble(1, 4)
    x = np.random.default_rng(1).standard_normal(64)
    x -= x.mean()
    assert learned.loss(A, x, x) == 0.0
    assert abs(learned.loss(A, x, np.zeros_like(x)) - 1.0) < 1e-15


def test_bf16_rounding_ties_to_even():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to the even mantissa (1.0)
    assert learned.bf16(1.0 + 2.0 ** -8) == 1.0
    assert learned.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert learned.bf16(1.0 + 2.0 ** -7) == 1.0 + 2.0 ** -7
    assert learned.bf16(-3.0) == -3.0


@pytest.mark.parametrize("kind", ["energy", "residual"])
def test_loss_gradient_matches_central_differences(kind):
    """The loss gradient through A and the net, by central differences of the loss itself."""
    q, n = 2, 2
    A = op.assemble(q, n).toarray()
    N = q * n
    dinv = (1.0 / np.diag(A)).reshape(N, N, N)
    rng = np.random.default_rng(40)
    r = rng.standard_normal(N ** 3)
    r -= r.mean()
    e = np.linalg.lstsq(A, r, rcond=None)[0]
    r, e = r.reshape(N, N, N), e.reshape(N, N, N)
    w = _rand_weights(41)
    val, g = learned.loss_and_gradient(w, A, dinv, r, e, kind, emulate_bf16=False)

    def f(ww):
        et, _ = learned.correction(ww, r, dinv, emulate_bf16=False)
        return learned.loss(A, e, et) if kind == "energy" else learned.residual_loss(A, r, et)

    assert abs(val - f(w)) <= 1e-12 * abs(val)
    h = 1e-6
    for i in rng.choice(len(w), 30, replace=False):
        ei = np.zeros_like(w)
        ei[i] = h
        fd = (f(w + ei) - f(w - ei)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_losses_at_exact_and_zero_corrections():
    q, n = 1, 4
    A = op.assemble(q, n)
    r = np.random.default_rng(5).standard_normal(64)
    r -= r.mean()
    e = np.linalg.lstsq(A.toarray(), r, rcond=None)[0]
    assert learned.residual_loss(A, r, np.zeros_like(r)) == 1.0
    assert learned.residual_loss(A, r, e) < 1e-24
    assert learned.loss(A, e, e) == 0.0
