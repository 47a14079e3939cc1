"""Oracle: reference forward and backward pass of the kernel-surrogate MLP.

The network maps four standardised chirp-time features of a (reference,
neighbour) pair to 128 reals (the real and imaginary parts of 64 basis
coefficients of the pair's analytic ratio kernel):

    a0 = x                                   [B, 4]
    a1 = gelu(a0 W1^T + b1)                  [B, 256]
    a2 = gelu(a1 W2^T + b2)                  [B, 256]
    a3 = gelu(a2 W3^T + b3)                  [B, 256]
    y  = a3 W4^T + b4                        [B, 128]
    L  = mean over all B * 128 entries of (y - t)^2

gelu(u) = u Phi(u) = u (1 + erf(u / sqrt 2)) / 2 (exact form), so
gelu'(u) = Phi(u) + u phi(u), phi the standard normal density.
Parameters are packed in one vector in the order W1, b1, W2, b2, W3, b3, W4,
b4 with W row-major [out][in].  Everything is float64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

LAYERS = ((4, 256), (256, 256), (256, 256), (256, 128))


def n_params() -> int:
    return sum(i * o + o for i, o in LAYERS)


def unpack(theta: np.ndarray):
    out, k = [], 0
    for i, o in LAYERS:
        W = theta[k:k + i * o].reshape(o, i)
        k += i * o
        b = theta[k:k + o]
        k += o
        out.append((W, b))
    return out


def gelu(u):
    return 0.5 * u * (1.0 + erf(u / math.sqrt(2.0)))


def gelu_grad(u):
    return 0.5 * (1.0 + erf(u / math.sqrt(2.0))) + u * np.exp(-0.5 * u * u) / math.sqrt(2.0 * math.pi)


def forward(theta, x):
    """Output y and the pre-activations / activations needed by backward."""
    layers = unpack(theta)
    acts, pres = [x], []
    a = x
    for li, (W, b) in enumerate(layers):
        u = a @ W.T + b
        pres.append(u)
        a = gelu(u) if li < len(layers) - 1 else u
        acts.append(a)
    return a, (acts, pres)


def loss(theta, x, t):
    y, _ = forward(theta, x)
    return float(np.mean((y - t) ** 2))


def grad(theta, x, t):
    """Loss and its gradient with respect to the packed parameters."""
    layers = unpack(theta)
    y, (acts, pres) = forward(theta, x)
    d = 2.0 * (y - t) / y.size                        # dL/dy
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        if li < len(layers) - 1:
            d = d * gelu_grad(pres[li])               # through the activation
        gW = d.T @ acts[li]
        gb = d.sum(axis=0)
        grads.append((gW, gb))
        d = d @ W                                     # to the layer input
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return float(np.mean((y - t) ** 2)), flat


def adam_step(theta, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, arXiv 1412.6980, Algorithm 1; step counts
    from 1): exponential moving averages of g and g^2, each divided by its bias
    factor 1 - beta^step; returns new theta, m, v."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def cosine_lr(lr0, k, total):
    """Learning rate of step k (0-based) of a cosine decay from lr0 to 0 over
    `total` steps: lr0 (1 + cos(pi k / total)) / 2."""
    return lr0 * 0.5 * (1.0 + math.cos(math.pi * k / total))


def train(theta, x, t, order, lr0):
    """Training as the surrogate does it: for step k = 0 .. steps-1 the rows
    order[k] of (x, t) form the batch, the gradient of the mean squared error
    is taken there, and Adam (moments starting at zero) moves theta with the
    cosine-decayed rate of step k.  Returns the final theta and the loss of
    every step (before its update)."""
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    hist = []
    steps = len(order)
    for k in range(steps):
        rows = np.asarray(order[k])
        L, g = grad(theta, x[rows], t[rows])
        hist.append(L)
        theta, m, v = adam_step(theta, g, m, v, k + 1, cosine_lr(lr0, k, steps))
    return theta, np.array(hist)
