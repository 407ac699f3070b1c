"""Element-local MLP of the learned PCG initial guess (not part of the
paper's method; it only changes the initial guess, and PCG always follows to
the same tolerance).

Network (per row = one element and one solution component, n = (P+1)^d
nodal values):
    z1 = W1 x + b1,  a1 = relu(z1)
    z2 = W2 a1 + b2, a2 = relu(z2)
    y  = W3 a2 + b3
Loss over a batch of B rows: L = 1/(2B) sum_rows |y - t|^2.
Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
    theta -= lr * (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps).
Flat parameter layout: W1 (H x n, row-major [out][in]), b1 (H), W2 (H x H),
b2 (H), W3 (n x H), b3 (n).

Initial weights: SplitMix64 (Vigna), the k-th output (k = 0, 1, ...) of a
generator seeded with s being mix(s + (k+1) * 0x9E3779B97F4A7C15); a weight of
a layer with fan-in f is (2u - 1) sqrt(6 / f), u = (output >> 11) * 2^-53;
biases start at 0.

The BF16 forward pass rounds weights and layer inputs to bfloat16
(round-to-nearest-even) and accumulates in FP32.
"""
import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
MASK = (1 << 64) - 1


def splitmix64(seed, k):
    z = (seed + (k + 1) * GOLDEN) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def sizes(n, H):
    return [(H, n), (H,), (H, H), (H,), (n, H), (n,)]


def n_params(n, H):
    return sum(int(np.prod(s)) for s in sizes(n, H))


def init_params(n, H, seed):
    """Flat FP64 parameter vector, in the order of the layout above."""
    out = np.zeros(n_params(n, H))
    k = 0
    pos = 0
    for shp in sizes(n, H):
        cnt = int(np.prod(shp))
        if len(shp) == 2:
            fan_in = shp[1]
            sc = np.sqrt(6.0 / fan_in)
            for i in range(cnt):
                u = (splitmix64(seed, k) >> 11) * (2.0 ** -53)
                out[pos + i] = (2.0 * u - 1.0) * sc
                k += 1
        pos += cnt
    return out


def unpack(theta, n, H):
    parts = []
    pos = 0
    for shp in sizes(n, H):
        cnt = int(np.prod(shp))
        parts.append(theta[pos:pos + cnt].reshape(shp))
        pos += cnt
    return parts


def bf16(a):
    """Round float32 values to bfloat16 (round to nearest, ties to even),
    returned as float32."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = (u + 0x7FFF + lsb) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32)


def forward(theta, X, n, H, dtype=np.float64, bf16_weights=False):
    W1, b1, W2, b2, W3, b3 = [p.astype(dtype) for p in unpack(theta, n, H)]
    X = X.astype(dtype)
    q = (lambda a: bf16(a)) if bf16_weights else (lambda a: a)
    z1 = q(X) @ q(W1).T + b1
    a1 = np.maximum(z1, 0)
    z2 = q(a1) @ q(W2).T + b2
    a2 = np.maximum(z2, 0)
    y = q(a2) @ q(W3).T + b3
    return y, (X, z1, a1, z2, a2)


def loss_and_grad(theta, X, T, n, H, dtype=np.float64):
    """L and dL/dtheta (flat), by the chain rule written out layer by layer."""
    W1, b1, W2, b2, W3, b3 = [p.astype(dtype) for p in unpack(theta, n, H)]
    y, (X, z1, a1, z2, a2) = forward(theta, X, n, H, dtype)
    B = X.shape[0]
    diff = y - T.astype(dtype)
    L = 0.5 * np.sum(diff * diff) / B
    dy = diff / B
    dW3 = dy.T @ a2
    db3 = dy.sum(axis=0)
    da2 = dy @ W3
    dz2 = da2 * (z2 > 0)
    dW2 = dz2.T @ a1
    db2 = dz2.sum(axis=0)
    da1 = dz2 @ W2
    dz1 = da1 * (z1 > 0)
    dW1 = dz1.T @ X
    db1 = dz1.sum(axis=0)
    g = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])
    return L, g


class Adam:
    def __init__(self, size, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, dtype=np.float64):
        self.m = np.zeros(size, dtype=dtype)
        self.v = np.zeros(size, dtype=dtype)
        self.k = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.dtype = dtype

    def step(self, theta, g):
        dt = self.dtype
        self.k += 1
        b1, b2 = dt(self.b1), dt(self.b2)
        self.m = b1 * self.m + (dt(1) - b1) * g
        self.v = b2 * self.v + (dt(1) - b2) * g * g
        mh = self.m / (dt(1) - b1 ** self.k)
        vh = self.v / (dt(1) - b2 ** self.k)
        return theta - dt(self.lr) * mh / (np.sqrt(vh) + dt(self.eps))
