"""Pins of the FP64 reference of the learned proposal (oracle/mlp.py) to
mathematics rather than to itself: central differences for the gradients,
the closed form of Adam's first steps, a hand-solvable forward pass, the +-1
structure of the projection and the sketch's estimate of the kink-test value
Phi(0) of the paper's score [Alg. 2, function D]."""
import numpy as np
import pytest

import oracle
import oracle.mlp as mlp
import synth


def rand_params(rng, scale=0.3):
    return rng.normal(0, scale, mlp.NPARAM)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = rand_params(rng, 0.2)
    phi = rng.normal(0, 1, (6, mlp.PHI))
    y = rng.normal(0, 1, 6)
    loss, g = mlp.loss_and_grad(p, phi, y)
    idx = np.concatenate([rng.choice(mlp.NPARAM, 300, replace=False),
                          np.arange(mlp.NPARAM - 129, mlp.NPARAM)])   # w3 and b3 in full
    h = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (mlp.loss_and_grad(pp, phi, y)[0] - mlp.loss_and_grad(pm, phi, y)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_adam_first_steps_closed_form():
    """With a constant gradient the bias-corrected moments are g and g^2, so
    every step moves each parameter by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    p0 = rng.normal(0, 1, 50)
    g = rng.normal(0, 1, 50)
    m = np.zeros(50)
    v = np.zeros(50)
    p = p0.copy()
    lr = 1e-3
    for t in (1, 2, 3):
        p, m, v = mlp.adam_step(p, g, m, v, t, lr)
        want = p0 - t * lr * g / (np.abs(g) + mlp.ADAM_EPS)
        assert np.allclose(p, want, rtol=0, atol=1e-12)


def test_forward_special_case():
    """W1 selects feature k into unit 0, W2 = identity, w3 = e_0: the output
    is max(phi_k, 0) + b3; phi = [s_i s_j, |s_i - s_j|, s_i + s_j]."""
    rng = np.random.default_rng(2)
    S = rng.normal(0, 1, (5, mlp.S_DIM))
    I, J = np.array([0, 1, 2, 3]), np.array([4, 3, 0, 1])
    phi = mlp.pair_features(S, I, J)
    for k, ref in [(5, S[I, 5] * S[J, 5]), (64 + 7, np.abs(S[I, 7] - S[J, 7])),
                   (128 + 63, S[I, 63] + S[J, 63])]:
        W1 = np.zeros((mlp.PHI, mlp.H1))
        W1[k, 0] = 1.0
        p = mlp.pack(W1, np.zeros(mlp.H1), np.eye(mlp.H1), np.zeros(mlp.H2),
                     np.eye(mlp.H2)[0], 0.25)
        out, _ = mlp.forward(p, phi)
        assert np.allclose(out, np.maximum(ref, 0) + 0.25, rtol=0, atol=1e-14)


def test_projection_is_pm1_from_the_counter_generator():
    P = mlp.projection(40, seed=3)
    assert set(np.unique(P)) <= {-1.0, 1.0}
    # column norms are exact for +-1 entries: |P e_k|^2 = 28
    assert np.all((P * P).sum(0) == mlp.D)
    for d, m in [(0, 0), (5, 17), (27, 39)]:
        top = oracle.ctr(3, 7, d, m) >> 63
        assert P[d, m] == (-1.0 if top else 1.0)


def test_sketch_estimates_the_kink_test_value():
    """sum_d s_i[d] s_j[d] - s_i[28+d] s_j[28+d] has expectation
    (56/M) Phi_ij(0) over P; across the pairs of C1 at W = 0 it must track
    the oracle's own Phi(0) (an independent computation in oracle.cpp).  With
    28 projections its noise is ~|x_i| |r_j| / sqrt(28), several times the
    spread of Phi(0) over unrelated pairs, so the correlation is moderate
    (0.37 here); a sign or index mistake in either half drives it to ~0."""
    w = synth.config("C1")
    lam = oracle.default_lambda(w.X, "ising")
    O = oracle.Oracle(w.X, "ising", lam)
    ei, ej, wv, th = O.get_model()
    S = mlp.sketch("ising", w.X, O.fields(), th, ei, ej, wv, seed=0)
    I, J = np.triu_indices(w.N, 1)
    est = ((S[I, :28] * S[J, :28]).sum(1) - (S[I, 28:56] * S[J, 28:56]).sum(1)) * w.M / 56.0
    phi = np.array([O.pair_deriv(i, j, 0.0) for i, j in zip(I, J)])
    c = np.corrcoef(est, phi)[0, 1]
    assert c > 0.25, c
    # statistics block
    assert np.allclose(S[:, 56], w.X.mean(1))
    assert np.allclose(S[:, 61], 0) and np.allclose(S[:, 62], 0)
    assert np.allclose(S[:, 63], th)


def test_sketch_statistics_closed_forms():
    """The statistics block against values the model fixes: at W = 0 with
    theta fitted (Ising: tanh theta_i = xbar_i) every field equals theta_i, so
    mean t = xbar, var t = 0, mean |h| = |atanh xbar|, mean r^2 = 1 - xbar^2
    (r = x - xbar), no degree and no coupling mass; after setting a known W,
    the degree and |W| columns count that W's entries per node (both ends)."""
    w = synth.ising_er(12, 300, 3.0, 0.4, 0.1, seed=31)
    O = oracle.Oracle(w.X, "ising", 1.0)
    ei, ej, wv, th = O.get_model()
    S = mlp.sketch("ising", w.X, O.fields(), th, ei, ej, wv, seed=0)
    xb = w.X.astype(float).mean(1)
    assert np.allclose(S[:, 57], xb, atol=1e-12)
    assert np.allclose(S[:, 58], 0, atol=1e-12)
    assert np.allclose(S[:, 59], np.abs(np.arctanh(xb)), atol=1e-12)
    assert np.allclose(S[:, 60], 1 - xb ** 2, atol=1e-12)
    I = np.array([0, 0, 3], np.int32)
    J = np.array([5, 7, 5], np.int32)
    V = np.array([0.5, -0.25, 0.125])
    O.set_model(I, J, V, th)
    ei, ej, wv, th = O.get_model()
    S = mlp.sketch("ising", w.X, O.fields(), th, ei, ej, wv, seed=0)
    deg = np.zeros(12)
    mass = np.zeros(12)
    for a, b, v in [(0, 5, 0.5), (0, 7, 0.25), (3, 5, 0.125)]:
        deg[[a, b]] += 1
        mass[[a, b]] += v
    assert np.allclose(S[:, 61], np.log1p(deg)) and np.allclose(S[:, 62], mass)
    # with couplings the fields vary across samples: var t > 0 on coupled nodes
    assert np.all(S[[0, 3, 5, 7], 58] > 0) and np.allclose(S[[1, 2], 58], 0, atol=1e-12)


def test_sketch_noise_is_the_projection_limit():
    """The sketch's estimate of Phi(0) is as good as 28 random +-1 projections
    allow, and no better: over the pairs of C1 at W = 0 its correlation with
    the exact Phi(0) equals the one predicted from the projection noise (the
    variance of the estimator over independent projection draws, computed
    here with numpy's generator, not the library's), within 0.08; the same
    estimator with 1024 projections per half would correlate above 0.85.  So
    the proposal's ranking is limited by what 64 numbers per node can carry
    about a pair, while the kink test that the residual screen evaluates
    from 1 B per sample ranks the pairs exactly."""
    w = synth.config("C1")
    lam = oracle.default_lambda(w.X, "ising")
    O = oracle.Oracle(w.X, "ising", lam)
    ei, ej, wv, th = O.get_model()
    H = O.fields()
    S = mlp.sketch("ising", w.X, H, th, ei, ej, wv, seed=0)
    I, J = np.triu_indices(w.N, 1)
    est = ((S[I, :28] * S[J, :28]).sum(1) - (S[I, 28:56] * S[J, 28:56]).sum(1)) * w.M / 56.0
    phi = np.array([O.pair_deriv(i, j, 0.0) for i, j in zip(I, J)])
    measured = np.corrcoef(est, phi)[0, 1]
    x = w.X.astype(np.float64)
    r = x - np.tanh(H)

    def draws(D, n, seed):
        """n independent estimates per pair with D projections per half."""
        rng = np.random.default_rng(seed)
        out = []
        for _ in range(n):
            P = rng.choice([-1.0, 1.0], size=(D, w.M))
            u, v = (x + r) @ P.T, (x - r) @ P.T
            out.append(((u[I] * u[J]).sum(1) - (v[I] * v[J]).sum(1)) / (2.0 * D))
        return np.array(out)

    E = draws(28, 48, 5)
    assert abs(E.mean(0) - phi).max() < 6 * np.sqrt(E.var(0).max() / 48)   # unbiased
    noise = E.var(0).mean()
    predicted = phi.std() / np.sqrt(phi.var() + noise)
    assert abs(measured - predicted) <= 0.08, (measured, predicted)
    wide = np.corrcoef(draws(1024, 1, 6)[0], phi)[0, 1]
    assert wide > 0.85, wide
    print(f"sketch vs Phi(0): measured {measured:.3f}, predicted {predicted:.3f}, 1024 projections {wide:.3f}")
