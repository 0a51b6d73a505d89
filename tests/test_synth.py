"""Checks of the seeded workload generators (not of the method)."""
import itertools

import numpy as np

import synth


def test_gibbs_moments_match_enumeration():
    """Gibbs samples of a small Ising model reproduce <x_i> and <x_i x_j> of the
    exact distribution P(x) ~ exp(sum_{i<j} W_ij x_i x_j + theta . x) within 4 sigma."""
    N = 6
    ei = np.array([0, 1, 2, 3, 0], np.int32)
    ej = np.array([1, 2, 3, 4, 5], np.int32)
    w = np.array([0.5, -0.4, 0.3, 0.6, -0.2])
    theta = np.array([0.1, -0.2, 0.0, 0.3, -0.1, 0.2])
    M = 4000
    X = synth.gibbs(N, M, ei, ej, w, theta, burn=50, thin=3, seed=1).astype(float)
    W = np.zeros((N, N))
    W[ei, ej] = w
    W[ej, ei] = w
    states = np.array(list(itertools.product([-1, 1], repeat=N)), float)
    logp = 0.5 * np.einsum("si,ij,sj->s", states, W, states) + states @ theta
    p = np.exp(logp - logp.max())
    p /= p.sum()
    mean = p @ states
    corr = np.einsum("s,si,sj->ij", p, states, states)
    m_hat = X.mean(1)
    c_hat = X @ X.T / M
    # thinning keeps samples nearly independent; allow 4 sigma with a 2x margin
    # for the remaining autocorrelation
    se = 2 * np.sqrt((1 - mean ** 2) / M)
    assert np.all(np.abs(m_hat - mean) < 4 * se + 1e-12)
    se2 = 2 * np.sqrt(np.clip(1 - corr ** 2, 0, None) / M) + 1e-12
    assert np.all(np.abs(c_hat - corr) < 4 * se2)


def test_glauber_transition_frequencies():
    """Parallel Glauber: P(x_{i,t+1} = 1 | x_t) = (1 + tanh h_{i,t}) / 2."""
    N, T = 3, 20000
    dst = np.array([0, 1, 2], np.int32)
    src = np.array([1, 2, 0], np.int32)
    w = np.array([0.8, -0.5, 0.3])
    X = synth.glauber(N, T, dst, src, w, np.zeros(N), seed=2).astype(float)
    for i, j, wij in zip(dst, src, w):
        for b in (-1, 1):
            sel = X[j, :-1] == b
            freq = (X[i, 1:][sel] == 1).mean()
            p = (1 + np.tanh(wij * b)) / 2
            assert abs(freq - p) < 4 * np.sqrt(p * (1 - p) / sel.sum())


def test_gauss_covariance():
    N, M = 5, 20000
    ei = np.array([0, 1, 2], np.int32)
    ej = np.array([1, 2, 3], np.int32)
    off = np.array([0.2, -0.15, 0.1])
    X, diag = synth.gauss(N, M, ei, ej, off, eps=0.1, seed=3)
    Theta = np.diag(diag)
    Theta[ei, ej] = off
    Theta[ej, ei] = off
    C = np.linalg.inv(Theta)
    Ch = X.astype(float) @ X.T.astype(float) / M
    assert np.abs(Ch - C).max() < 6 * np.sqrt(np.outer(np.diag(C), np.diag(C)) * 2 / M).max()


def test_graphs_and_determinism():
    ei, ej = synth.er_undirected(2000, 3.0, seed=0)
    assert np.all(ei < ej)
    assert abs(len(ei) - 3000) < 5 * np.sqrt(3000)
    ei2, ej2 = synth.er_undirected(2000, 3.0, seed=0)
    assert np.array_equal(ei, ei2) and np.array_equal(ej, ej2)
    a, b = synth.regular(1000, 3, seed=0)
    deg = np.bincount(np.concatenate([a, b]), minlength=1000)
    assert np.all(deg == 3)
    assert len(set(zip(a.tolist(), b.tolist()))) == len(a)
    d, s = synth.er_directed(2000, 5.0, seed=0)
    assert np.all(d != s)
    assert abs(len(d) - 10000) < 5 * np.sqrt(10000)


def test_gauss_scaling_recipe():
    """The runtime study's problems: ER mean degree 5, off-diagonal precisions
    ~ N(-1000, 10^2), diagonal sum_j |W_ij| / (1 - eps)^2, M = 10 samples."""
    w = synth.gauss_scaling(4000, 10, seed=3)
    N = w.N
    assert w.X.shape == (N, 10) and w.X.dtype == np.float32 and np.all(np.isfinite(w.X))
    assert abs(2 * len(w.ei) / N - 5.0) < 0.3
    assert abs(w.w.mean() + 1000.0) < 1.0 and abs(w.w.std() - 10.0) < 0.5
    deg_abs = np.zeros(N)
    np.add.at(deg_abs, w.ei, np.abs(w.w))
    np.add.at(deg_abs, w.ej, np.abs(w.w))
    has = deg_abs > 0
    assert np.allclose(w.theta[has], deg_abs[has] / (1 - 1e-3) ** 2)
