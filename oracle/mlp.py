"""FP64 reference of the learned proposal: per-node sketches, the symmetric
pair feature, the 3-layer ranking MLP, its loss, gradients and Adam step.

TEST INFRASTRUCTURE ONLY: used by ``tests/`` (never by the GPU library).  The
proposal is not part of the paper; it ranks the candidate pairs of the
second-neighbour search [Alg. 4] so that only the most promising ones get the
exact score d(i, j) [Alg. 2, function D], which stays the judge of every
accepted edge.  Definitions (the GPU library implements the same ones in its
own kernels):

* Sketch of node i, 64 values.  With x_i the input-side samples, y_i the
  targets (Ising: y = x; kinetic: x_{i,t+1}; Gaussian: y = x), t_i = tanh h_i
  and r_i = y_i - t_i (Gaussian: r_i = the residual of the pseudolikelihood,
  t_i := r_i), and P in {+-1}^{28 x M} with P[d, m] = +1 unless the top bit of
  SplitMix64 ctr(seed, 7, d, m) is set:
    s[0:28]  = P (x_i + r_i) / sqrt(M),   s[28:56] = P (x_i - r_i) / sqrt(M),
    s[56:64] = mean y, mean t, var t, mean |h| (Gaussian: mean |r|), mean r^2,
               log(1 + deg_i), sum_j |W_ij|, theta_i.
  Since E[P^T P] = 28 I, sum_d (s_i[d] s_j[d] - s_i[28+d] s_j[28+d]) has
  expectation (56 / M) (x_i . r_j + r_i . x_j): the kink-test value Phi(0) of
  the pair, which the first layer can read off the elementwise products.
* Pair feature phi(s_i, s_j) = [s_i * s_j, |s_i - s_j|, s_i + s_j] (192).
* MLP: z1 = phi W1 + b1, h1 = relu(z1) (128); z2 = h1 W2 + b2, h2 = relu(z2)
  (128); out = h2 . w3 + b3.  Target: log(1 + gain).  Loss: mean (out - y)^2 / 2.
* Adam (Kingma & Ba 2015): beta1 = 0.9, beta2 = 0.999, eps = 1e-8, with bias
  correction.

Flat parameter order (float32 on the GPU): W1 [192][128] (input-major), b1,
W2 [128][128], b2, w3, b3.

Pins: ``tests/test_oracle_pins.py`` checks the gradients against central
differences, the first Adam step against its closed form, the forward pass
against a hand-solvable special case and the projection's +-1 structure.
"""
from __future__ import annotations

import numpy as np

D = 28
S_DIM = 64
PHI = 192
H1 = 128
H2 = 128
STREAM_PROJ = 7
NPARAM = PHI * H1 + H1 + H1 * H2 + H2 + H2 + 1

ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def projection(M: int, seed: int) -> np.ndarray:
    """P[d, m] in {+-1}: -1 when the top bit of ctr(seed, 7, d, m) is set."""
    from . import ctr
    P = np.empty((D, M), np.float64)
    for d in range(D):
        for m in range(M):
            P[d, m] = -1.0 if (ctr(seed, STREAM_PROJ, d, m) >> 63) else 1.0
    return P


def sketch(model: str, X: np.ndarray, H: np.ndarray, theta: np.ndarray,
           ei: np.ndarray, ej: np.ndarray, w: np.ndarray, seed: int) -> np.ndarray:
    """Sketches (N x 64) at the state given by the fields H (N x M, the
    oracle's ``fields()``), theta and the nonzero couplings (ei, ej, w)."""
    N = X.shape[0]
    if model == "kinetic":
        x = X[:, :-1].astype(np.float64)
        y = X[:, 1:].astype(np.float64)
    else:
        x = X.astype(np.float64)
        y = x
    M = x.shape[1]
    if model == "gauss":
        r = H.astype(np.float64)
        t = r
        habs = np.abs(r)
    else:
        t = np.tanh(H)
        r = y - t
        habs = np.abs(H)
    P = projection(M, seed)
    S = np.zeros((N, S_DIM))
    S[:, 0:D] = (x + r) @ P.T / np.sqrt(M)
    S[:, D:2 * D] = (x - r) @ P.T / np.sqrt(M)
    S[:, 56] = y.mean(1)
    S[:, 57] = t.mean(1)
    S[:, 58] = (t * t).mean(1) - t.mean(1) ** 2
    S[:, 59] = habs.mean(1)
    S[:, 60] = (r * r).mean(1)
    deg = np.zeros(N)
    l1 = np.zeros(N)
    for a, b, v in zip(ei, ej, w):
        if v == 0:
            continue
        deg[a] += 1
        l1[a] += abs(v)
        if model != "kinetic":
            deg[b] += 1
            l1[b] += abs(v)
    S[:, 61] = np.log1p(deg)
    S[:, 62] = l1
    S[:, 63] = theta
    return S


def pair_features(S: np.ndarray, I, J) -> np.ndarray:
    a, b = S[np.asarray(I)], S[np.asarray(J)]
    return np.concatenate([a * b, np.abs(a - b), a + b], axis=1)


def unpack(p: np.ndarray):
    p = np.asarray(p, np.float64)
    o = 0
    W1 = p[o:o + PHI * H1].reshape(PHI, H1); o += PHI * H1
    b1 = p[o:o + H1]; o += H1
    W2 = p[o:o + H1 * H2].reshape(H1, H2); o += H1 * H2
    b2 = p[o:o + H2]; o += H2
    w3 = p[o:o + H2]; o += H2
    b3 = p[o]; o += 1
    assert o == NPARAM
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]])


def forward(p: np.ndarray, phi: np.ndarray):
    W1, b1, W2, b2, w3, b3 = unpack(p)
    z1 = phi @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    out = h2 @ w3 + b3
    return out, (phi, z1, h1, z2, h2)


def loss_and_grad(p: np.ndarray, phi: np.ndarray, y: np.ndarray):
    """Loss mean (out - y)^2 / 2 and its gradient (flat, same order as p)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    out, (phi, z1, h1, z2, h2) = forward(p, phi)
    B = phi.shape[0]
    dout = (out - y) / B
    loss = 0.5 * np.mean((out - y) ** 2)
    gw3 = h2.T @ dout
    gb3 = dout.sum()
    dz2 = np.outer(dout, w3) * (z2 > 0)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2.T) * (z1 > 0)
    gW1 = phi.T @ dz1
    gb1 = dz1.sum(0)
    return loss, pack(gW1, gb1, gW2, gb2, gw3, gb3)


def adam_step(p, g, m, v, t, lr):
    """One Adam step (t = 1 for the first); returns (p, m, v)."""
    m = ADAM_B1 * m + (1 - ADAM_B1) * g
    v = ADAM_B2 * v + (1 - ADAM_B2) * g * g
    mh = m / (1 - ADAM_B1 ** t)
    vh = v / (1 - ADAM_B2 ** t)
    return p - lr * mh / (np.sqrt(vh) + ADAM_EPS), m, v
