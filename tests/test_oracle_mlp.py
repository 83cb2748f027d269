"""Pins of the FP64 reference MLP (CPU): finite differences and BF16 rounding."""
import numpy as np

from oracle import mlp_ref as R


def _setup(n=40, seed=0):
    rng = np.random.default_rng(seed)
    p = rng.normal(size=R.NP) * 0.3
    X = rng.normal(size=(n, R.NIN))
    base = rng.uniform(0.1, 1.0, n)
    target = base * rng.uniform(1.0, 1.5, n)
    scale = np.maximum(target, 0.05)
    return p, X, base, target, scale


def test_gradient_matches_central_differences():
    p, X, base, target, scale = _setup()
    loss, g = R.loss_and_grad(p, X, base, target, scale, bf16=False)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(np.arange(R.OW1, R.OB1), 8), rng.choice(np.arange(R.OW2, R.OB2), 16),
                          rng.choice(np.arange(R.OW3, R.OB3), 6), [R.OB1 + 3, R.OB2 + 5, R.OB3]])
    for i in idx:
        h = 1e-6 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (R.loss_and_grad(pp, X, base, target, scale, bf16=False)[0]
              - R.loss_and_grad(pm, X, base, target, scale, bf16=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (i, fd, g[i])


def test_bf16_rounding_known_values():
    x = np.array([1.0, 1.00390625, 1.005859375, 3.0, -2.5, 1e-40, 65504.0])
    r = R.bf16_round(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: rounds to even (1.0)
    assert r[0] == 1.0 and r[1] == 1.0
    assert r[2] == 1.0078125  # above the tie: rounds up
    assert r[3] == 3.0 and r[4] == -2.5
    assert r[6] == 65536.0


def test_prediction_never_below_chord():
    p, X, base, target, scale = _setup()
    d, _ = R.forward(p, X, base)
    assert np.all(d >= base)
