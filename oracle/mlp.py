"""Numpy reference of the warm-start network (oracle; test infrastructure
only).  Not a passage of the paper: the network is this project's learned
warm start of the self-consistency loop.

Network: L fully connected layers, y = W_L h_{L-1} + b_L with
h_l = tanh(W_l h_{l-1} + b_l), h_0 = x; loss = mean over the batch of the sum
of squared output errors.  Parameters are packed layer by layer as
[W_1 (out x in, row-major), b_1, W_2, b_2, ...] in float64 here.

Adam (Kingma & Ba, 2015): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
p <- p - lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
"""
import numpy as np


def layer_shapes(d_in, width, depth, d_out):
    dims = [d_in] + [width] * (depth - 1) + [d_out]
    return [(dims[i + 1], dims[i]) for i in range(depth)]


def n_params(shapes):
    return sum(o * i + o for o, i in shapes)


def unpack(p, shapes):
    out = []
    k = 0
    for o, i in shapes:
        w = p[k:k + o * i].reshape(o, i)
        k += o * i
        b = p[k:k + o]
        k += o
        out.append((w, b))
    return out


def round_bf16(a):
    """Round float32 values to bfloat16 (8-bit significand), to nearest with ties
    to even, returned as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p, shapes, x, bf16=False):
    """Returns the output and the list of layer activations (for backward).
    bf16: both operands of every layer product are rounded to bfloat16 first
    (activations as float32 values), products summed exactly."""
    acts = [x]
    h = x
    layers = unpack(p, shapes)
    for li, (w, b) in enumerate(layers):
        if bf16:
            z = round_bf16(h) @ round_bf16(w).T + b
        else:
            z = h @ w.T + b
        h = np.tanh(z) if li < len(layers) - 1 else z
        acts.append(h)
    return h, acts


def loss_and_grad(p, shapes, x, t):
    """Mean-squared loss (sum over outputs, mean over rows) and its gradient
    with respect to the packed parameters, by backpropagation."""
    y, acts = forward(p, shapes, x)
    nb = x.shape[0]
    loss = float(np.sum((y - t) ** 2) / nb)
    layers = unpack(p, shapes)
    grads = []
    d = 2.0 * (y - t) / nb
    for li in range(len(layers) - 1, -1, -1):
        w, b = layers[li]
        if li < len(layers) - 1:
            d = d * (1.0 - acts[li + 1] ** 2)
        gw = d.T @ acts[li]
        gb = d.sum(axis=0)
        grads.append((gw, gb))
        d = d @ w
    g = []
    for gw, gb in reversed(grads):
        g.append(gw.ravel())
        g.append(gb)
    return loss, np.concatenate(g)


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


_M64 = (1 << 64) - 1


def splitmix64(z):
    """SplitMix64 output for state z (Steele, Lea & Flood 2014): the state is
    advanced by the golden-ratio increment, then mixed."""
    z = (z + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def minibatch_rows(seed, step, batch, rows):
    """Rows of minibatch `step`: slot q takes SplitMix64(seed * 0xD1B54A32D192ED03
    + step * batch + q) mod rows (sampling with replacement)."""
    base = (seed * 0xD1B54A32D192ED03) & _M64
    return np.array([splitmix64((base + step * batch + q) & _M64) % rows
                     for q in range(batch)])


def train(p, shapes, x, t, batch, steps, lr, seed):
    """Adam steps on sampled minibatches; returns the parameters and the loss
    of each minibatch before its step."""
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    losses = []
    for s in range(steps):
        r = minibatch_rows(seed, s, batch, x.shape[0])
        loss, g = loss_and_grad(p, shapes, x[r], t[r])
        losses.append(loss)
        p, m, v = adam_step(p, g, m, v, s + 1, lr)
    return p, np.array(losses)
