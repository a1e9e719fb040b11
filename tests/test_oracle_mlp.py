"""Pin for the FP64 MLP reference: gradients vs central finite differences."""
import numpy as np


def _params(rng):
    shapes = [(16, 64), (64,), (64, 64), (64,), (64, 4), (4,)]
    return [rng.normal(scale=0.3, size=s) for s in shapes]


def test_mlp_gradients_finite_differences(orc):
    rng = np.random.default_rng(0)
    P = _params(rng)
    x = rng.normal(size=(32, 16))
    y = rng.integers(0, 4, size=32)
    loss, grads = orc.mlp_loss_grad(P, x, y)
    h = 1e-6
    for pi, (p, g) in enumerate(zip(P, grads)):
        flat = p.reshape(-1)
        for idx in rng.choice(flat.size, min(flat.size, 12), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = orc.mlp_loss_grad(P, x, y)
            flat[idx] = old - h
            lm, _ = orc.mlp_loss_grad(P, x, y)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g.reshape(-1)[idx]) <= 1e-7 * max(1.0, abs(fd)), (pi, idx)


def test_mlp_loss_of_uniform_logits(orc):
    rng = np.random.default_rng(1)
    P = [np.zeros(s) for s in [(16, 64), (64,), (64, 64), (64,), (64, 4), (4,)]]
    loss, _ = orc.mlp_loss_grad(P, rng.normal(size=(8, 16)), rng.integers(0, 4, 8))
    assert abs(loss - np.log(4.0)) < 1e-15
