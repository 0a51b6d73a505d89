"""The gain bounds behind the Ising / kinetic screening contraction, checked
on the CPU against the oracle's exact gains.

For a pair with no coupling yet, f'(0) = a and the curvature of the smooth
part is a sum of sech^2 terms bracketed by c e^{-2|w|} and c e^{2|w|}, c its
value at w = 0.  With e = |a| - lambda and q = 2e/c the best gain of the
L1-penalised step [Alg. 2, function D] lies in
    [(c/4)((1+q) ln(1+q) - q),  (c/4)(q + (1-q) ln(1-q))]   (upper: q < 1)
and is 0 when |a| <= lambda.  The screen keeps every pair whose upper bound
reaches a threshold taken from the lower bounds, so both sides must hold for
every pair, at W = 0 and at states with W != 0.
"""
import numpy as np
import pytest

import oracle
import synth


def phi(q):
    return (1 + q) * np.log1p(q) - q


def psi(q):
    return np.where(q < 1, q + (1 - q) * np.log1p(-np.minimum(q, 0.999999999)), np.inf)


def curvatures(O, model):
    T = np.tanh(O.fields())
    return (1.0 - T * T).sum(axis=1)


@pytest.mark.parametrize("model", ["ising", "kinetic"])
def test_gain_bounds_hold(model):
    if model == "ising":
        w = synth.ising_er(50, 300, 3.0, 0.5, 0.3, seed=21)
    else:
        w = synth.kinetic_er(50, 300, 4.0, 0.5, seed=22)
    N = w.N
    lam = 0.5 * oracle.default_lambda(w.X, model)
    O = oracle.Oracle(w.X, model, lam)
    checked = 0
    for state in range(3):
        ei, ej, wv, _ = O.get_model()
        coupled = set(zip(ei.tolist(), ej.tolist())) if len(ei) else set()
        cv = curvatures(O, model)
        if model == "kinetic":
            I, J = [a.ravel() for a in np.meshgrid(np.arange(N), np.arange(N), indexing="ij")]
            keep = I != J
        else:
            I, J = np.triu_indices(N, 1)
            keep = np.ones(len(I), bool)
        I, J = I[keep].astype(np.int32), J[keep].astype(np.int32)
        free = np.array([(i, j) not in coupled and (model == "kinetic" or (j, i) not in coupled)
                         for i, j in zip(I.tolist(), J.tolist())])
        I, J = I[free], J[free]
        g, _ = O.score_pairs(I, J)
        a = np.array([O.pair_deriv(i, j, 0.0) for i, j in zip(I, J)])
        c = cv[I] if model == "kinetic" else cv[I] + cv[J]
        e = np.abs(a) - lam
        below = e <= 0
        assert np.all(g[below] <= 1e-12 * lam), model
        q = 2 * np.maximum(e, 0) / c
        lo = 0.25 * c * phi(q)
        up = 0.25 * c * psi(q)
        pos = ~below
        assert pos.sum() > 20
        tol = 1e-9 * np.maximum(1.0, g)
        assert np.all(lo[pos] <= g[pos] + tol[pos]), (state, np.max(lo[pos] - g[pos]))
        assert np.all(g[pos] <= up[pos] + tol[pos]), (state, np.max(g[pos] - up[pos]))
        # the bracket is tight for small steps: both ends agree to O(q)
        small = pos & (q < 0.05)
        if small.any():
            assert np.all(up[small] / np.maximum(lo[small], 1e-300) < 1 + 2 * q[small] + 1e-9)
        checked += pos.sum()
        O.gcd_sweep(N, "exhaustive")
    assert checked > 100


@pytest.mark.parametrize("model", ["ising", "kinetic"])
def test_gain_bound_of_current_couplings(model):
    """A coupling w0 != 0: with s = sign(w0) the step's penalty change is at
    least lambda s d, so gain <= (c/4) psi(2 |a - lambda s| / c) with a the
    derivative of the smooth part at w0 and c the curvature at the current
    fields.  Checked for every coupling after a few oracle sweeps."""
    if model == "ising":
        w = synth.ising_er(60, 300, 3.0, 0.5, 0.3, seed=23)
    else:
        w = synth.kinetic_er(60, 300, 4.0, 0.5, seed=24)
    lam = 0.5 * oracle.default_lambda(w.X, model)
    O = oracle.Oracle(w.X, model, lam)
    checked = 0
    for sweep in range(3):
        O.gcd_sweep(w.N // 2, "exhaustive")
        ei, ej, wv, _ = O.get_model()
        nz = wv != 0
        ei, ej, wv = ei[nz], ej[nz], wv[nz]
        cv = curvatures(O, model)
        g, _ = O.score_pairs(ei, ej)
        a = np.array([O.pair_deriv(i, j, v) for i, j, v in zip(ei, ej, wv)])
        c = cv[ei] if model == "kinetic" else cv[ei] + cv[ej]
        q = 2 * np.abs(a - lam * np.sign(wv)) / c
        up = 0.25 * c * psi(q)
        assert np.all(g <= up + 1e-9 * np.maximum(1.0, g)), (sweep, np.max(g - up))
        checked += len(g)
    assert checked > 30
