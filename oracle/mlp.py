"""FP64 forward and backward of the warm-start network, in numpy.

TEST INFRASTRUCTURE ONLY: the reference the GPU network kernels are checked
against.

The network (an added component; the paper has none): layer l maps
x -> z = x W_l^T + b_l, followed by SiLU(z) = z sigmoid(z) on every layer but
the last. Parameters are one flat vector, per layer W_l[out][in] row major and
then b_l[out]. The loss is the mean of the squared errors over all outputs
of the batch. Adam follows Kingma & Ba (2015) with bias-corrected moments.

The network is specified with BF16 operands and FP32 accumulation. The
optional ``operand`` argument of ``forward`` and ``backward`` is a rounding
applied to both factors of every matrix product (for example to BF16); the
products and sums themselves stay in FP64.
"""
import numpy as np


def unpack(p, dims):
    out, o = [], 0
    for l in range(len(dims) - 1):
        din, dout = dims[l], dims[l + 1]
        W = p[o:o + din * dout].reshape(dout, din)
        o += din * dout
        b = p[o:o + dout]
        o += dout
        out.append((W, b))
    assert o == p.size
    return out


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def _identity(a):
    return a


def forward(p, dims, x, operand=None):
    """Returns the output and the cache (pre-activations and layer inputs)."""
    op = operand or _identity
    layers = unpack(np.asarray(p, dtype=np.float64), dims)
    h = np.asarray(x, dtype=np.float64)
    cache = []
    for l, (W, b) in enumerate(layers):
        z = op(h) @ op(W).T + b
        cache.append((h, z))
        h = z * sigmoid(z) if l < len(layers) - 1 else z
    return h, cache


def mse(y, t):
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(p, dims, cache, dy, operand=None):
    """Gradient of the loss with respect to the flat parameters, given dy =
    d loss / d output."""
    op = operand or _identity
    layers = unpack(np.asarray(p, dtype=np.float64), dims)
    grads = [None] * len(layers)
    dz = np.asarray(dy, dtype=np.float64)
    for l in range(len(layers) - 1, -1, -1):
        W, b = layers[l]
        h, z = cache[l]
        grads[l] = (op(dz).T @ op(h), dz.sum(axis=0))
        if l > 0:
            dh = op(dz) @ op(W)
            zp = cache[l - 1][1]
            s = sigmoid(zp)
            dz = dh * (s * (1.0 + zp * (1.0 - s)))
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def loss_and_grad(p, dims, x, t):
    y, cache = forward(p, dims, x)
    loss, dy = mse(y, t)
    return loss, backward(p, dims, cache, dy)


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
