"""FP64 reference of the surrogate's operations (numpy).

TEST INFRASTRUCTURE ONLY (part of the oracle).  Each function is the plain
definition of the operation:
  periodic 3x3x3 convolution  Y[co,p] = b[co] + sum_{ci,t} W[co,ci,t] X[ci, p + off(t)]
  weight gradient             dW[co,ci,t] = sum_p dY[co,p] X[ci, p + off(t)]
  data gradient               dX[ci,q] = sum_{co,t} W[co,ci,t] dY[co, q - off(t)]
  2x2x2 average pooling, nearest 2x upsampling, masked mean squared error and
  the Adam update (Kingma & Ba 2015).
Tap t = 9 dz + 3 dy + dx with offsets dz-1, dy-1, dx-1 along (z, y, x).
Shifts are np.roll (periodic); channel sums are tensordot.
"""
from __future__ import annotations

import numpy as np


def offsets():
    return [(t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1) for t in range(27)]


def shifted(X, off):
    """X[..., p + off] with periodic wrap, X shaped (C, D, H, W)."""
    dz, dy, dx = off
    return np.roll(X, shift=(-dz, -dy, -dx), axis=(1, 2, 3))


def conv(X, W, b=None, relu=False, skip=None):
    Y = np.zeros((W.shape[0],) + X.shape[1:])
    for t, off in enumerate(offsets()):
        Y += np.tensordot(W[:, :, t], shifted(X, off), axes=(1, 0))
    if b is not None:
        Y += b[:, None, None, None]
    if relu:
        Y = np.maximum(Y, 0.0)
    if skip is not None:
        Y = Y + skip
    return Y


def wgrad(X, dY):
    dW = np.zeros((dY.shape[0], X.shape[0], 27))
    for t, off in enumerate(offsets()):
        dW[:, :, t] = np.tensordot(dY, shifted(X, off), axes=([1, 2, 3], [1, 2, 3]))
    return dW


def dgrad(W, dY):
    dX = np.zeros((W.shape[1],) + dY.shape[1:])
    for t, (dz, dy, dx) in enumerate(offsets()):
        dX += np.tensordot(W[:, :, t], shifted(dY, (-dz, -dy, -dx)), axes=(0, 0))
    return dX


def pool(X):
    C, D, H, W = X.shape
    return X.reshape(C, D // 2, 2, H // 2, 2, W // 2, 2).mean(axis=(2, 4, 6))


def up(X):
    return X.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def mse(Y, T, mask):
    m = mask.sum()
    L = (mask[None] * (Y - T) ** 2).sum() / (Y.shape[0] * m)
    dY = 2.0 * mask[None] * (Y - T) / (Y.shape[0] * m)
    return L, dY


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    p = p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return p, m, v
