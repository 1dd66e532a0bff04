"""FP64 reference of the learned smoothness indicator (test infrastructure only).

The indicator is a project extension that sits beside the paper's WENO5
reconstruction (Sec. 3.2): a small multilayer perceptron looks at a 5-cell
stencil along one direction and predicts whether WENO5's nonlinear weights
would stay at their ideal values there.  Cells it calls smooth take the
linear fifth-order stencil (the ideal-weight limit of WENO5) for every
variable of that direction; all others take full WENO5.

Definitions followed here, and by nothing else in this package:
  * inputs (15): for alpha1, rho = a1r1 + a2r2 and p, the 5 stencil values
    minus the centre value, divided by max(max_j |v_j - v_centre|, sqrt(eps));
    every input lies in [-1, 1] and the centre input is 0;
  * network: 15 -> 32 -> 32 -> 1, tanh-form GELU on both hidden layers,
    logistic sigmoid on the output; P(smooth) = sigmoid(z);
  * loss: mean binary cross-entropy; optimiser: Adam;
  * label: smooth iff the largest |omega_r - d_r| over the three stencils,
    both faces and all reconstructed variables is below 0.01 (the WENO5
    weights of the oracle's `weno5`).
"""
from __future__ import annotations

import math

import numpy as np

import oracle

NIN, NH = 15, 32
GELU_C = math.sqrt(2.0 / math.pi)


# ------------------------------------------------------------------ features

def features(alpha, rho, p, eps=1e-6):
    """alpha, rho, p: arrays [..., 5] of stencil values -> [..., 15] inputs."""
    out = []
    floor = math.sqrt(eps)
    for v in (alpha, rho, p):
        v = np.asarray(v, dtype=np.float64)
        d = v - v[..., 2:3]
        scale = np.maximum(np.abs(d).max(axis=-1, keepdims=True), floor)
        out.append(d / scale)
    return np.concatenate(out, axis=-1)


def label(stencils, eps=1e-6, threshold=0.01):
    """stencils: [nvar, 5] primitive values of one cell along one direction.
    1 if every reconstructed variable keeps its WENO5 weights within
    `threshold` of the ideal ones (both faces), else 0."""
    dev = max(oracle.weno5(stencils[v], eps)[2] for v in range(stencils.shape[0]))
    return int(dev < threshold)


# ------------------------------------------------------------------- network

def init_params(seed=0):
    """Glorot-uniform weights, zero biases, from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)

    def glorot(n_in, n_out):
        a = math.sqrt(6.0 / (n_in + n_out))
        return rng.uniform(-a, a, size=(n_in, n_out))

    return {"W1": glorot(NIN, NH), "b1": np.zeros(NH), "W2": glorot(NH, NH), "b2": np.zeros(NH),
            "W3": glorot(NH, 1), "b3": np.zeros(1)}


def gelu(x):
    """GELU in its tanh form: x/2 (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3)))."""
    return 0.5 * x * (1.0 + np.tanh(GELU_C * (x + 0.044715 * x ** 3)))


def gelu_grad(x):
    t = np.tanh(GELU_C * (x + 0.044715 * x ** 3))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * 0.044715 * x * x)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(params, X):
    """X [N, 15] -> (P(smooth) [N], cache for backward)."""
    Z1 = X @ params["W1"] + params["b1"]
    H1 = gelu(Z1)
    Z2 = H1 @ params["W2"] + params["b2"]
    H2 = gelu(Z2)
    z = (H2 @ params["W3"] + params["b3"])[:, 0]
    return sigmoid(z), (X, Z1, H1, Z2, H2, z)


def bce(P, y):
    P = np.clip(P, 1e-15, 1.0 - 1e-15)
    return float(-np.mean(y * np.log(P) + (1.0 - y) * np.log(1.0 - P)))


def loss_and_grads(params, X, y):
    """Mean BCE and its gradient with respect to every parameter."""
    P, (X, Z1, H1, Z2, H2, z) = forward(params, X)
    n = X.shape[0]
    dz = (sigmoid(z) - y) / n                    # d(mean BCE)/dz
    g = {"W3": H2.T @ dz[:, None], "b3": np.array([dz.sum()])}
    dH2 = dz[:, None] @ params["W3"].T
    dZ2 = dH2 * gelu_grad(Z2)
    g["W2"], g["b2"] = H1.T @ dZ2, dZ2.sum(axis=0)
    dH1 = dZ2 @ params["W2"].T
    dZ1 = dH1 * gelu_grad(Z1)
    g["W1"], g["b1"] = X.T @ dZ1, dZ1.sum(axis=0)
    return bce(P, y), g


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; state holds m, v and the step count t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = b1 * m + (1.0 - b1) * grads[k]
        v[...] = b2 * v + (1.0 - b2) * grads[k] ** 2
        mhat = m / (1.0 - b1 ** t)
        vhat = v / (1.0 - b2 ** t)
        params[k] -= lr * mhat / (np.sqrt(vhat) + eps)
    return params
