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


def hand_net():
    """A 16-64-64-4 network whose outputs follow by hand (every weight is a
    small dyadic number, exact in BF16 and FP32).  Layer 1 splits each input
    into its positive part (units 0..15) and negative part (units 16..31) and
    adds a constant unit 32 (bias 1) and a dead unit 33 (bias -1).  Layer 2
    sums the positive parts (unit 0), the negative parts (unit 1), doubles
    the constant (unit 2) and forms relu(0.5 - relu(x0)) (unit 3); unit 4 has
    bias -3 and dies.  Layer 3 (no ReLU) reads
      logit0 = P - 0.5 N, logit1 = N, logit2 = 2 - 5, logit3 = h3 + 0.25.
    A ReLU after the output layer, a missing hidden ReLU, or W read in the
    transposed layout changes at least one logit."""
    W1 = np.zeros((16, 64)); b1 = np.zeros(64)
    for i in range(16):
        W1[i, i] = 1.0
        W1[i, 16 + i] = -1.0
    b1[32], b1[33] = 1.0, -1.0
    W2 = np.zeros((64, 64)); b2 = np.zeros(64)
    W2[:16, 0] = 1.0
    W2[16:32, 1] = 1.0
    W2[32, 2] = 2.0
    W2[33, 2] = 7.0          # reads the dead unit: contributes only if its ReLU is missing
    W2[0, 3] = -1.0
    b2[3] = 0.5
    b2[4] = -3.0
    W3 = np.zeros((64, 4)); b3 = np.array([0.0, 0.0, -5.0, 0.25])
    W3[0, 0], W3[1, 0], W3[1, 1], W3[2, 2], W3[3, 3], W3[4, 1] = 1.0, -0.5, 1.0, 1.0, 1.0, 9.0
    return [W1, b1, W2, b2, W3, b3]


def hand_logits(x):
    P = np.maximum(x, 0.0).sum(1)
    N = np.maximum(-x, 0.0).sum(1)
    h3 = np.maximum(0.5 - np.maximum(x[:, 0], 0.0), 0.0)
    return np.stack([P - 0.5 * N, N, np.full(len(x), -3.0), h3 + 0.25], 1)


HAND_X = np.array([[1.0, -2.0, 0.5, -0.25] + [0.0] * 11 + [3.0],
                   [0.25, 0.0, -1.0] + [0.0] * 12 + [-4.0],
                   [-0.5] * 16], np.float64)


def test_mlp_forward_hand_values(orc):
    logits, _ = orc.mlp_forward(hand_net(), HAND_X)
    want = hand_logits(HAND_X)
    assert np.array_equal(logits, want), (logits, want)
    # spelled out for the first row: P = 4.5, N = 2.25, h3 = 0
    assert logits[0].tolist() == [3.375, 2.25, -3.0, 0.25]
    assert logits[1].tolist() == [0.25 - 2.5, 5.0, -3.0, 0.5]
