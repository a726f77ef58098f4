"""Reference of the warm-start network in plain numpy, FP64 (test
infrastructure: the GPU forward / backward / Adam kernels are checked
against it, and it is checked against finite differences).

Network (the learned part of the static workflow: a map from the external
potential to the self-consistent potentials and chemical potential, used as
the initial guess of the fixed-point iteration):

    x  : [B, 1, H, W]   normalised V_ext
    h1 = relu(conv3(x;  W1, b1))        C channels
    h2 = relu(conv3(h1; W2, b2))        C channels
    h3 = relu(conv3(h2; W3, b3))        C channels
    maps = conv1(h3; Wm, bm)            2 channels: normalised (U, Delta)
    mu   = mean_{H,W}(h3) . wmu + bmu   scalar

conv3 is a 3x3 convolution with periodic padding (the lattice is periodic),
conv1 a pointwise channel mix.  Loss:
    L = mean((maps - Y)^2) + lam_mu * mean((mu - y_mu)^2).
Parameters are kept in one flat vector in the order
W1 b1 W2 b2 W3 b3 Wm bm wmu bmu; W of a conv3 is [Cout, Cin, 3, 3].
"""
import numpy as np


def shapes(C):
    return [("W1", (C, 1, 3, 3)), ("b1", (C,)), ("W2", (C, C, 3, 3)), ("b2", (C,)),
            ("W3", (C, C, 3, 3)), ("b3", (C,)), ("Wm", (2, C)), ("bm", (2,)), ("wmu", (C,)), ("bmu", (1,))]


def nparams(C):
    return sum(int(np.prod(s)) for _, s in shapes(C))


def unpack(theta, C):
    out, o = {}, 0
    for name, s in shapes(C):
        k = int(np.prod(s))
        out[name] = theta[o:o + k].reshape(s)
        o += k
    return out


def init_params(C, seed):
    """He-normal weights from a seeded PCG64 stream, zero biases."""
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for name, s in shapes(C):
        if name.startswith("b"):
            parts.append(np.zeros(s))
        else:
            fan_in = int(np.prod(s[1:])) if len(s) > 1 else s[0]
            parts.append(g.standard_normal(s) * np.sqrt(2.0 / fan_in))
    return np.concatenate([p.ravel() for p in parts])


def conv3(x, W, b):
    """y[n, o, i, j] = b[o] + sum_{c, di, dj} W[o, c, di, dj] x[n, c, i+di-1, j+dj-1] (periodic)."""
    y = np.zeros((x.shape[0], W.shape[0]) + x.shape[2:])
    for di in range(3):
        for dj in range(3):
            xs = np.roll(x, shift=(1 - di, 1 - dj), axis=(2, 3))  # xs[i, j] = x[i + di - 1, j + dj - 1]
            y += np.einsum("oc,ncij->noij", W[:, :, di, dj], xs)
    return y + b[None, :, None, None]


def conv3_backward(x, W, gy):
    """Gradients of conv3 w.r.t. its input, weights and bias."""
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for di in range(3):
        for dj in range(3):
            xs = np.roll(x, shift=(1 - di, 1 - dj), axis=(2, 3))
            gW[:, :, di, dj] = np.einsum("noij,ncij->oc", gy, xs)
            gxs = np.einsum("oc,noij->ncij", W[:, :, di, dj], gy)
            gx += np.roll(gxs, shift=(di - 1, dj - 1), axis=(2, 3))
    gb = gy.sum(axis=(0, 2, 3))
    return gx, gW, gb


def forward(theta, x, C):
    p = unpack(theta, C)
    z1 = conv3(x, p["W1"], p["b1"]); h1 = np.maximum(z1, 0)
    z2 = conv3(h1, p["W2"], p["b2"]); h2 = np.maximum(z2, 0)
    z3 = conv3(h2, p["W3"], p["b3"]); h3 = np.maximum(z3, 0)
    maps = np.einsum("kc,ncij->nkij", p["Wm"], h3) + p["bm"][None, :, None, None]
    g = h3.mean(axis=(2, 3))
    mu = g @ p["wmu"] + p["bmu"][0]
    cache = (x, z1, h1, z2, h2, z3, h3, g)
    return maps, mu, cache


def loss_and_grad(theta, x, Y, ymu, C, lam_mu=1.0):
    """L and dL/dtheta (flat, parameter order of `shapes`)."""
    p = unpack(theta, C)
    maps, mu, (x, z1, h1, z2, h2, z3, h3, g) = forward(theta, x, C)
    nm, nb = maps.size, mu.size
    L = np.sum((maps - Y) ** 2) / nm + lam_mu * np.sum((mu - ymu) ** 2) / nb
    gmaps = 2.0 * (maps - Y) / nm
    gmu = 2.0 * lam_mu * (mu - ymu) / nb
    gWm = np.einsum("nkij,ncij->kc", gmaps, h3)
    gbm = gmaps.sum(axis=(0, 2, 3))
    gwmu = g.T @ gmu
    gbmu = np.array([gmu.sum()])
    HW = h3.shape[2] * h3.shape[3]
    gh3 = np.einsum("kc,nkij->ncij", p["Wm"], gmaps) + (gmu[:, None] * p["wmu"][None, :] / HW)[:, :, None, None]
    gz3 = gh3 * (z3 > 0)
    gh2, gW3, gb3 = conv3_backward(h2, p["W3"], gz3)
    gz2 = gh2 * (z2 > 0)
    gh1, gW2, gb2 = conv3_backward(h1, p["W2"], gz2)
    gz1 = gh1 * (z1 > 0)
    _, gW1, gb1 = conv3_backward(x, p["W1"], gz1)
    grads = dict(W1=gW1, b1=gb1, W2=gW2, b2=gb2, W3=gW3, b3=gb3, Wm=gWm, bm=gbm, wmu=gwmu, bmu=gbmu)
    return L, np.concatenate([grads[n].ravel() for n, _ in shapes(C)])


def adam_step(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments); returns (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
