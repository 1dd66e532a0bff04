"""FP64 reference of the learned smoothness indicator (test infrastructure only).

The indicator is a project extension that sits beside the paper's WENO5
reconstruction (Sec. 3.2): a small multilayer perceptron looks at a 5-cell
stencil along one direction and predicts whether WENO5's nonlinear weights
would stay at their ideal values there.  Cells it calls smooth take the
linear fifth-order stencil (the ideal-weight limit of WENO5) for every
variable of that direction; all others take full WENO5.

Definitions followed here (the GPU kernels implement the same definitions
independently):
  * inputs (15): for alpha1, rho = a1r1 + a2r2 and p, the 5 stencil values
    minus the centre value, divided by max(max_j |v_j - v_centre|, sqrt(eps));
    every input lies in [-1, 1] and the centre input is 0;
  * network: 15 -> 32 -> 32 -> 1, tanh-form GELU on both hidden layers,
    logistic sigmoid on the output; P(smooth) = sigmoid(z);
  * loss: mean binary cross-entropy; optimiser: Adam;
  * label: smooth iff the largest |omega_r - d_r| over the three stencils,
    both faces and all reconstructed variables is below 0.01 (the WENO5
    weights of the oracle's `weno5`);
  * number formats of the GPU form: the operands of every matrix product
    (inputs, W1, W2, the hidden activations H1, the back-propagated dZ2 and
    dZ1) are rounded to bfloat16 (nearest, ties to even); products
    accumulate in FP32; biases, W3, the output layer, GELU and its
    derivative, and all other element-wise work are FP32; the master
    weights and Adam moments are FP32.  `forward(..., bf16=True)` and
    `loss_and_grads(..., bf16=True)` round at exactly those points and do
    the rest in FP64, so they differ from the GPU only by FP32 rounding;
  * routing: a (cell, direction) whose P(smooth) exceeds tau takes the
    linear stencil for every variable and both of its faces.
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


def bf16(x):
    """Round to the nearest bfloat16 value (8 significant bits, ties to
    even), returned as float64.  Values stay far inside bfloat16's exponent
    range here, so no overflow or subnormal handling is needed."""
    m, e = np.frexp(np.asarray(x, dtype=np.float64))
    return np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)


def _id(x):
    return x


def forward(params, X, bf16_operands=False):
    """X [N, 15] -> (P(smooth) [N], cache for backward)."""
    r = bf16 if bf16_operands else _id
    Xr = r(X)
    Z1 = Xr @ r(params["W1"]) + params["b1"]
    H1 = gelu(Z1)
    H1r = r(H1)
    Z2 = H1r @ r(params["W2"]) + params["b2"]
    H2 = gelu(Z2)
    z = (H2 @ params["W3"] + params["b3"])[:, 0]
    return sigmoid(z), (Xr, Z1, H1r, Z2, H2, z)


def bce(P, y):
    P = np.clip(P, 1e-15, 1.0 - 1e-15)
    return float(-np.mean(y * np.log(P) + (1.0 - y) * np.log(1.0 - P)))


def loss_and_grads(params, X, y, bf16_operands=False):
    """Mean BCE and its gradient with respect to every parameter.  With
    bf16_operands the matrix-product operands are rounded as the GPU form
    defines (see the module docstring); the bias gradients sum the unrounded
    values."""
    r = bf16 if bf16_operands else _id
    P, (Xr, Z1, H1r, Z2, H2, z) = forward(params, X, bf16_operands)
    n = X.shape[0]
    dz = (sigmoid(z) - y) / n                    # d(mean BCE)/dz
    g = {"W3": H2.T @ dz[:, None], "b3": np.array([dz.sum()])}
    dH2 = dz[:, None] @ params["W3"].T
    dZ2 = dH2 * gelu_grad(Z2)
    dZ2r = r(dZ2)
    g["W2"], g["b2"] = H1r.T @ dZ2r, dZ2.sum(axis=0)
    dH1 = dZ2r @ r(params["W2"]).T
    dZ1 = dH1 * gelu_grad(Z1)
    g["W1"], g["b1"] = Xr.T @ r(dZ1), dZ1.sum(axis=0)
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


# ------------------------------------------------------- flat parameter order

ORDER = (("W1", (NIN, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH, 1)), ("b3", (1,)))
NPARAM = sum(int(np.prod(shape)) for _, shape in ORDER)   # 1601


def flatten(params):
    """Parameters in the flat order W1 (in-major), b1, W2 (in-major), b2, W3, b3."""
    return np.concatenate([np.asarray(params[k], dtype=np.float64).reshape(-1) for k, _ in ORDER])


def unflatten(flat):
    out, o = {}, 0
    for k, shape in ORDER:
        n = int(np.prod(shape))
        out[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shape).copy()
        o += n
    return out


# ------------------------------------------------------------- whole fields

_AXIS = {0: 3, 1: 2, 2: 1}  # direction -> axis of a [v, z, y, x] array


def _stencils(spec, a, d, lo, hi):
    """5-cell stencils along direction d of a padded scalar field a [z, y, x],
    for interior-relative cells lo..hi-1 along d and interior cells along the
    other active directions: array [..., 5] in the field's axis order."""
    ax = _AXIS[d] - 1
    sl = [slice(None)] * 3
    for e in range(spec.ndim):
        if e != d:
            sl[_AXIS[e] - 1] = slice(3, 3 + spec.n[e])
    out = []
    for t in range(5):
        s2 = list(sl)
        s2[ax] = slice(3 + lo - 2 + t, 3 + hi - 2 + t)
        out.append(a[tuple(s2)])
    return np.stack(out, axis=-1)


def field_features(spec, w, d, lo=0, hi=None):
    """Features [..., 15] of cells lo..hi-1 along direction d from a padded
    primitive field w [nv, z, y, x]."""
    hi = spec.n[d] if hi is None else hi
    nv = spec.nvar
    alpha = _stencils(spec, w[nv - 1], d, lo, hi)
    rho = _stencils(spec, w[0] + w[1], d, lo, hi)
    p = _stencils(spec, w[nv - 2], d, lo, hi)
    return features(alpha, rho, p, spec.weno_eps)


def harvest(spec, q):
    """(features [ndim * cells, 15], labels [ndim * cells], max deviation)
    of every interior (cell, direction), samples ordered direction-major,
    then z, y, x; q is a conservative state with ghosts filled."""
    w, st = oracle.cons_to_prim_field(spec, q)
    assert st == oracle.OK
    X, Y, D = [], [], []
    nv = spec.nvar
    for d in range(spec.ndim):
        f = field_features(spec, w, d)
        sts = np.stack([_stencils(spec, w[v], d, 0, spec.n[d]) for v in range(nv)], axis=-2)  # [..., nv, 5]
        X.append(f.reshape(-1, NIN))
        flat = sts.reshape(-1, nv, 5)
        dev = np.array([max(oracle.weno5(c[v], spec.weno_eps)[2] for v in range(nv)) for c in flat])
        D.append(dev)
        Y.append((dev < 0.01).astype(np.uint8))
    return np.concatenate(X), np.concatenate(Y), np.concatenate(D)


def smooth_probability(spec, q, params, bf16_operands=True):
    """P(smooth) of every reconstruction cell (-1 .. n along each direction,
    interior along the others) as an array [ndim, *padded shape] (NaN where
    no reconstruction happens); q with ghosts filled."""
    w, _ = oracle.cons_to_prim_field(spec, q)
    P = np.full((spec.ndim,) + spec.shape[1:], np.nan)
    for d in range(spec.ndim):
        f = field_features(spec, w, d, -1, spec.n[d] + 1)
        prob, _ = forward(params, f.reshape(-1, NIN), bf16_operands)
        sl = [slice(None)] * 3
        for e in range(spec.ndim):
            sl[_AXIS[e] - 1] = slice(3, 3 + spec.n[e]) if e != d else slice(2, 4 + spec.n[d])
        P[(d,) + tuple(sl)] = prob.reshape(f.shape[:-1])
    return P


def rhs_learned(spec, q, params, tau, bf16_operands=True):
    """(right-hand side with routed reconstruction, status, P): q with ghosts
    filled; a (cell, direction) with P > tau takes the linear stencil."""
    P = smooth_probability(spec, q, params, bf16_operands)
    mask = np.ascontiguousarray(np.nan_to_num(P, nan=0.0) > tau, dtype=np.uint8)
    L, st = oracle.rhs(spec, q, oracle.RECON_MASK, mask)
    return L, st, P


def run_learned(spec, q, params, tau, nsteps, cfl, bf16_operands=True):
    """(q after nsteps SSP-RK3 steps with routed reconstruction, time, status,
    fraction of (cell, direction) reconstructions routed to the linear
    stencil); the step size comes from q^n as in the oracle's run."""
    q = np.array(q, dtype=np.float64)
    dxmin = min(spec.dx[:spec.ndim])
    t, smooth, total = 0.0, 0, 0
    for _ in range(nsteps):
        smax, st = oracle.max_wavespeed(spec, q)
        if st != oracle.OK:
            return q, t, st, smooth / max(total, 1)
        dt = cfl * dxmin / smax
        q0, qs = q.copy(), q.copy()
        for stage in (1, 2, 3):
            qs = oracle.fill_ghosts(spec, qs)
            L, st, P = rhs_learned(spec, qs, params, tau, bf16_operands)
            if st != oracle.OK:
                return q, t, st, smooth / max(total, 1)
            ok = ~np.isnan(P)
            smooth += int((P[ok] > tau).sum())
            total += int(ok.sum())
            qs = oracle.rk3_combine(stage, q0, qs, L, dt)
        q = qs
        t += dt
    return q, t, oracle.OK, smooth / max(total, 1)
