"""Weight-seeding network, plain fp64 reference (TEST INFRASTRUCTURE).

Only the test-suite may import this module. It is the definition the GPU kernels of the
seeding model are checked against; it shares no code with them.

Network (a learned start for the weight iteration of Sec. II, not part of the paper): 81
inputs (L/12, 16 frustration statistics, a 64-bin energy histogram of a T = 2 canonical
run), normalized per input as (x - mean) / sd; three hidden layers of 128 with GELU,
gelu(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2; 256 linear outputs, the estimate of
[S(E) - S(E_top)]/N on the grid e_j = -2 + 2j/255. Loss: masked mean squared error,
L = sum m (y - t)^2 / sum m. Optimizer: Adam (Kingma and Ba, ICLR 2015) with bias correction.

Parameter vector (float, this order, weights row-major [in][out]):
  W0 [96 x 128] (input rows 81..95 are padding, zero), b0 [128], W1 [128 x 128], b1 [128],
  W2 [128 x 128], b2 [128], W3 [128 x 256], b3 [256].
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

D_IN, D_PAD, HID, D_OUT = 81, 96, 128, 256
SHAPES = [("W0", (D_PAD, HID)), ("b0", (HID,)), ("W1", (HID, HID)), ("b1", (HID,)),
          ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (HID, D_OUT)), ("b3", (D_OUT,))]
N_PARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], np.float64).reshape(shp)
        o += n
    return out


def flatten(P):
    return np.concatenate([np.asarray(P[name], np.float64).reshape(-1) for name, _ in SHAPES])


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    # d/dz [z Phi(z)] = Phi(z) + z phi(z)
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def normalize(X, norm):
    """X [B, 81] -> [B, 96]: (x - mean)/sd on the 81 inputs, zeros in the padding."""
    mean, sd = norm[0], norm[1]
    Xn = np.zeros((X.shape[0], D_PAD))
    Xn[:, :D_IN] = (np.asarray(X, np.float64) - mean) / sd
    return Xn


def forward(theta, norm, X, keep=False):
    P = unflatten(theta)
    A0 = normalize(X, norm)
    Z1 = A0 @ P["W0"] + P["b0"]
    A1 = gelu(Z1)
    Z2 = A1 @ P["W1"] + P["b1"]
    A2 = gelu(Z2)
    Z3 = A2 @ P["W2"] + P["b2"]
    A3 = gelu(Z3)
    Y = A3 @ P["W3"] + P["b3"]
    if keep:
        return Y, (A0, Z1, A1, Z2, A2, Z3, A3)
    return Y


def loss(theta, norm, X, T, M):
    Y = forward(theta, norm, X)
    return float(np.sum(M * (Y - T) ** 2) / np.sum(M))


def loss_and_grad(theta, norm, X, T, M):
    """Masked MSE and its gradient by the chain rule, layer by layer."""
    P = unflatten(theta)
    Y, (A0, Z1, A1, Z2, A2, Z3, A3) = forward(theta, norm, X, keep=True)
    msum = np.sum(M)
    L = float(np.sum(M * (Y - T) ** 2) / msum)
    dY = 2.0 * M * (Y - T) / msum
    G = {}
    G["W3"] = A3.T @ dY
    G["b3"] = dY.sum(axis=0)
    dZ3 = (dY @ P["W3"].T) * gelu_grad(Z3)
    G["W2"] = A2.T @ dZ3
    G["b2"] = dZ3.sum(axis=0)
    dZ2 = (dZ3 @ P["W2"].T) * gelu_grad(Z2)
    G["W1"] = A1.T @ dZ2
    G["b1"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ P["W1"].T) * gelu_grad(Z1)
    G["W0"] = A0.T @ dZ1
    G["b0"] = dZ1.sum(axis=0)
    return L, flatten(G)


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t >= 1 (in place on theta, m, v)."""
    m[:] = b1 * m + (1.0 - b1) * g
    v[:] = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    theta[:] = theta - lr * mh / (np.sqrt(vh) + eps)


def init_params(seed: int):
    """Glorot-uniform weights, zero biases, zero padding rows."""
    rng = np.random.default_rng(seed)
    P = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            fan_in = D_IN if name == "W0" else shp[0]
            a = math.sqrt(6.0 / (fan_in + shp[1]))
            w = rng.uniform(-a, a, shp)
            if name == "W0":
                w[D_IN:] = 0.0
            P[name] = w
        else:
            P[name] = np.zeros(shp)
    return flatten(P)
