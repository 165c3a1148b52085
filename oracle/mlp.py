"""Reference (fp64, numpy) of the learned priority's network and its gradient.

TEST INFRASTRUCTURE, part of the oracle.  The network is an MLP
8 -> 64 -> 64 -> 1 with GELU; GELU(x) = x/2 * (1 + T(sqrt(2/pi) * (x +
0.044715 x^3))), where T is the [7/6] Pade approximant of tanh (Lambert's
continued fraction), set to +-1 for |t| >= 4.97.  Training minimises the mean
squared error to a target.  Weights are one flat vector of 4801 values:
W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3.

The backward pass here is the exact derivative of this forward; the tests pin
it against central finite differences.
"""
import numpy as np

N_PARAMS = 4801
K = 0.7978845608
C3 = 0.044715
CUT = 4.97


def unpack(w):
    w = np.asarray(w, np.float64)
    return (w[:512].reshape(64, 8), w[512:576], w[576:4672].reshape(64, 64), w[4672:4736],
            w[4736:4800], w[4800])


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3, [b3]])


def tanh_pade(t):
    t = np.asarray(t, np.float64)
    t2 = t * t
    num = t * (135135.0 + t2 * (17325.0 + t2 * (378.0 + t2)))
    den = 135135.0 + t2 * (62370.0 + t2 * (3150.0 + t2 * 28.0))
    r = np.clip(num / den, -1.0, 1.0)
    return np.where(t >= CUT, 1.0, np.where(t <= -CUT, -1.0, r))


def tanh_pade_grad(t):
    t = np.asarray(t, np.float64)
    t2 = t * t
    num = t * (135135.0 + t2 * (17325.0 + t2 * (378.0 + t2)))
    den = 135135.0 + t2 * (62370.0 + t2 * (3150.0 + t2 * 28.0))
    dnum = 135135.0 + t2 * (51975.0 + t2 * (1890.0 + 7.0 * t2))
    dden = t * (124740.0 + t2 * (12600.0 + 168.0 * t2))
    g = (dnum * den - num * dden) / (den * den)
    inside = (np.abs(t) < CUT) & (np.abs(num / den) <= 1.0)
    return np.where(inside, g, 0.0)


def gelu(x):
    x = np.asarray(x, np.float64)
    return 0.5 * x * (1.0 + tanh_pade(K * (x + C3 * x ** 3)))


def gelu_grad(x):
    x = np.asarray(x, np.float64)
    t = K * (x + C3 * x ** 3)
    return 0.5 * (1.0 + tanh_pade(t)) + 0.5 * x * tanh_pade_grad(t) * K * (1.0 + 3.0 * C3 * x * x)


def forward(w, X):
    """Outputs y (B,) and the cache for backward."""
    W1, b1, W2, b2, W3, b3 = unpack(w)
    X = np.asarray(X, np.float64)
    h1 = X @ W1.T + b1
    a1 = gelu(h1)
    h2 = a1 @ W2.T + b2
    a2 = gelu(h2)
    y = a2 @ W3 + b3
    return y, (X, h1, a1, h2, a2)


def loss(w, X, t):
    y, _ = forward(w, X)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def grad(w, X, t):
    """Gradient of the mean squared error with respect to the 4801 weights."""
    W1, b1, W2, b2, W3, b3 = unpack(w)
    y, (X, h1, a1, h2, a2) = forward(w, X)
    B = len(y)
    dy = 2.0 * (y - np.asarray(t, np.float64)) / B
    dW3 = a2.T @ dy
    db3 = dy.sum()
    d2 = np.outer(dy, W3) * gelu_grad(h2)
    dW2 = d2.T @ a1
    db2 = d2.sum(0)
    d1 = (d2 @ W2) * gelu_grad(h1)
    dW1 = d1.T @ X
    db1 = d1.sum(0)
    return pack(dW1, db1, dW2, db2, dW3, db3)


def init(seed):
    """He-style initial weights (a reference; the GPU library has its own)."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((64, 8)) * np.sqrt(2.0 / 8)
    W2 = rng.standard_normal((64, 64)) * np.sqrt(2.0 / 64)
    W3 = rng.standard_normal(64) * np.sqrt(1.0 / 64)
    return pack(W1, np.zeros(64), W2, np.zeros(64), W3, 0.0)
