"""Warm start for the radiosity solve, CPU reference (TEST INFRASTRUCTURE ONLY).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark import this module; the product library never does and the two
share no code.  The paper has no counterpart: the warm start is an extension
around its Jacobi solve (section 3 / 5.1), where any starting guess B^0 is
allowed and only the iteration count changes.  Everything is FP64 numpy.

  * POD basis by the method of snapshots (Sirovich, Q. Appl. Math. 1987):
    Gram matrix G = S^T S of the snapshot columns, its eigenpairs
    G w_j = lambda_j w_j in decreasing order, modes phi_j = S w_j / sqrt(lambda_j),
    singular values sigma_j = sqrt(lambda_j).
  * Multilayer perceptron: hidden layers h_l = tanh(W_l h_{l-1} + b_l), linear
    output y = W_L h_{L-1} + b_L; parameters packed layer by layer as W_l
    (out x in, row-major) followed by b_l.
  * Loss (1 / 2B) sum_b sum_j w_j (y_bj - t_bj)^2 and its gradient by the
    chain rule (backpropagation).
  * Adam (Kingma and Ba, ICLR 2015), with bias-corrected moments.
  * Sun features: (cos azimuth, sin azimuth, elevation mapped linearly from
    [e_lo, e_hi] to [-1, 1]).
"""
from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------------------
# POD (method of snapshots)
def pod_basis(S: np.ndarray, m: int):
    """Modes Phi (N x m) and singular values sigma (m) of the snapshot matrix
    S (N x M, one snapshot per column)."""
    S = np.asarray(S, dtype=np.float64)
    G = S.T @ S
    lam, W = np.linalg.eigh(G)
    order = np.argsort(lam)[::-1][:m]
    lam, W = lam[order], W[:, order]
    sigma = np.sqrt(np.maximum(lam, 0.0))
    Phi = (S @ W) / sigma[None, :]
    return Phi, sigma


def pod_project(Phi: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Coefficients c = Phi^T B (m x R)."""
    return Phi.T @ B


def pod_expand(Phi: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Field Phi c (N x R)."""
    return Phi @ c


# ----------------------------------------------------------------------------
# multilayer perceptron
def param_count(sizes) -> int:
    return int(sum(sizes[l + 1] * sizes[l] + sizes[l + 1] for l in range(len(sizes) - 1)))


def unpack(params: np.ndarray, sizes):
    """Views (W_l, b_l) into the packed parameter vector."""
    out, off = [], 0
    for l in range(len(sizes) - 1):
        fi, fo = sizes[l], sizes[l + 1]
        W = params[off:off + fo * fi].reshape(fo, fi)
        off += fo * fi
        b = params[off:off + fo]
        off += fo
        out.append((W, b))
    return out


def mlp_forward(params: np.ndarray, sizes, X: np.ndarray, keep: bool = False):
    """Outputs (B x sizes[-1]) for inputs X (B x sizes[0]); with keep=True also
    the list of layer inputs [X, h_1, ..., h_{L-1}]."""
    h = np.asarray(X, dtype=np.float64)
    hs = [h]
    layers = unpack(np.asarray(params, dtype=np.float64), sizes)
    for l, (W, b) in enumerate(layers):
        z = h @ W.T + b
        h = np.tanh(z) if l < len(layers) - 1 else z
        if l < len(layers) - 1:
            hs.append(h)
    return (h, hs) if keep else h


def mlp_loss_grad(params: np.ndarray, sizes, X: np.ndarray, T: np.ndarray, w: np.ndarray):
    """Loss (1/2B) sum_b sum_j w_j (y_bj - t_bj)^2 and its gradient with respect
    to the packed parameters."""
    params = np.asarray(params, dtype=np.float64)
    Y, hs = mlp_forward(params, sizes, X, keep=True)
    B = X.shape[0]
    diff = Y - T
    loss = 0.5 * float(np.sum(w[None, :] * diff * diff)) / B
    delta = w[None, :] * diff / B                     # dL/dy
    layers = unpack(params, sizes)
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        h_in = hs[l]
        grads[l] = (delta.T @ h_in, delta.sum(axis=0))
        if l > 0:
            delta = (delta @ W) * (1.0 - h_in * h_in)    # tanh'(z) = 1 - tanh(z)^2
    g = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, g


class Adam:
    """Adam with bias correction: m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
    theta <- theta - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""

    def __init__(self, n: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, theta: np.ndarray, g: np.ndarray) -> np.ndarray:
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mh = self.m / (1.0 - self.b1 ** self.t)
        vh = self.v / (1.0 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)


def sun_features(suns: np.ndarray, e_lo: float = 5.0, e_hi: float = 30.0) -> np.ndarray:
    """(cos az, sin az, elevation scaled to [-1, 1]) for unit sun vectors."""
    s = np.asarray(suns, dtype=np.float64)
    az = np.arctan2(s[:, 1], s[:, 0])
    el = np.rad2deg(np.arcsin(np.clip(s[:, 2], -1.0, 1.0)))
    return np.column_stack([np.cos(az), np.sin(az), 2.0 * (el - e_lo) / (e_hi - e_lo) - 1.0])
