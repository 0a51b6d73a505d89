"""Gradient as distance [Appendix, "Gradient as distance"] on the GPU against
the FP64 oracle, through the C ABI: the pair distances, the NNDescent lists
and FindBest under that distance, and GCD sweeps whose E_best it ranks.

Tolerances as in test_gpu_parity.py (1e-10 relative in FP64 mode, 1e-4 in
FP32 mode; an absolute term of rtol * M * 1e-3)."""
import numpy as np
import pytest

import oracle
import synth
from tests.test_gpu_parity import RTOL, close, ctx_for, compare_lists

pytestmark = pytest.mark.gpu


def state(model, seed):
    if model == "ising":
        w = synth.ising_er(220, 300, 3.0, 0.4, 0.1, seed=seed)
    elif model == "kinetic":
        w = synth.kinetic_er(200, 300, 4.0, 0.3, seed=seed)
    else:
        w = synth.gauss_er(160, 200, 4.0, 0.2, seed=seed)
    lam = oracle.default_lambda(w.X, model)
    O = oracle.Oracle(w.X, model, lam)
    # couplings on (nearly) every row: both branches of the distance, and
    # sample-dependent fields, so distances carry no exact ties (a row
    # without couplings has one tanh value, and its pairs' distances then
    # repeat exactly)
    for _ in range(3):
        O.gcd_sweep(2 * w.N, "exhaustive")
    return w, lam, O


def oracle_dist(O, model):
    """The oracle's search score of an unordered pair under the gradient
    distance (kinetic: the larger of the two directions)."""
    def f(a, b):
        d = O.grad_pairs(np.array([a], np.int32), np.array([b], np.int32))[0]
        if model == "kinetic":
            d = max(d, O.grad_pairs(np.array([b], np.int32), np.array([a], np.int32))[0])
        return d
    return f


def gpu_at(O, w, lam, prec):
    ei, ej, wv, th = O.get_model()
    C = ctx_for(w, lam, prec)
    C.set_model(ei, ej, wv, th)
    return C


@pytest.mark.parametrize("model", ["ising", "kinetic", "gauss"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_grad_pairs_match_oracle(model, prec):
    w, lam, O = state(model, 3)
    C = gpu_at(O, w, lam, prec)
    rng = np.random.default_rng(1)
    I = rng.integers(0, w.N, 4000).astype(np.int32)
    J = rng.integers(0, w.N, 4000).astype(np.int32)
    keep = I != J
    I, J = I[keep], J[keep]
    ei, ej, _, _ = O.get_model()
    I = np.concatenate([I, ei]).astype(np.int32)     # every current coupling too
    J = np.concatenate([J, ej]).astype(np.int32)
    d = C.grad_pairs(I, J).cpu().numpy()
    do = O.grad_pairs(I, J)
    ok = close(d, do, RTOL[prec], w.M)
    assert ok.all(), (np.flatnonzero(~ok)[:5], d[~ok][:5], do[~ok][:5])
    if model != "kinetic":   # symmetric models: d(i,j) = d(j,i) bit for bit
        assert np.array_equal(d, C.grad_pairs(J, I).cpu().numpy())


def test_grad_pairs_reject_invalid():
    w, lam, O = state("ising", 3)
    C = gpu_at(O, w, lam, "fp64")
    with pytest.raises(Exception):
        C.grad_pairs(np.array([0, 5], np.int32), np.array([1, 5], np.int32))
    with pytest.raises(Exception):
        C.grad_pairs(np.array([0], np.int32), np.array([w.N], np.int32))
    assert len(C.grad_pairs(np.zeros(0, np.int32), np.zeros(0, np.int32))) == 0


@pytest.mark.parametrize("model", ["ising", "kinetic"])
def test_gradient_knn_lists_match_oracle(model):
    w, lam, O = state(model, 4)
    C = gpu_at(O, w, lam, "fp64")
    S = np.arange(w.N, dtype=np.int32)
    k = 6
    Jo, Go, it_o = O.knn(S, k, "nndescent", seed=0, level=0, dist="gradient")
    nbr, g, it = C.knn(S, k, 0, "nndescent", dist="gradient")
    compare_lists(nbr.cpu().numpy(), g.cpu().numpy(), Jo, Go, 1e-10, score=oracle_dist(O, model), S=S)
    assert it == it_o


@pytest.mark.parametrize("model", ["ising", "kinetic"])
def test_gradient_findbest_matches_oracle(model):
    w, lam, O = state(model, 5)
    C = gpu_at(O, w, lam, "fp64")
    m = 2 * w.N
    Io, Jo, Go, sto = O.find_best(m, "nndescent", seed=0, dist="gradient")
    I, J, G, st = C.find_best(m, "gradient")
    assert st["levels"] == sto["levels"]
    assert close(G.cpu().numpy(), Go, 1e-10, w.M).all()
    diff = set(zip(Io.tolist(), Jo.tolist())) ^ set(zip(I.cpu().numpy().tolist(), J.cpu().numpy().tolist()))
    # a pair in one result only must tie (by the oracle's own distance) with
    # the m-th distance: a swap at the boundary
    gm = Go[-1]
    for a, b in diff:
        da = O.grad_pairs(np.array([a], np.int32), np.array([b], np.int32))[0]
        assert abs(da - gm) <= 1e-9 * max(1.0, gm), (a, b, da, gm)
    # the distances returned are those of the pairs
    assert close(G.cpu().numpy(), O.grad_pairs(I.cpu().numpy(), J.cpu().numpy()), 1e-10, w.M).all()


@pytest.mark.parametrize("model", ["ising", "kinetic"])
def test_gradient_sweeps_track_oracle(model):
    """Sweeps whose E_best is ranked by the gradient distance (exact KNN, so
    both sides rank the same pairs): the same objective as the oracle's
    sweeps, and no sweep lowers it."""
    w = synth.ising_er(150, 300, 3.0, 0.4, 0.1, seed=7) if model == "ising" else \
        synth.kinetic_er(150, 300, 4.0, 0.3, seed=7)
    lam = oracle.default_lambda(w.X, model)
    O = oracle.Oracle(w.X, model, lam)
    C = ctx_for(w, lam, "fp64", kappa=1.0)
    prev = O.objective()
    for s in range(3):
        Io, Jo, _, _ = O.find_best(w.N, "exact_knn", dist="gradient")
        I, J, G, _ = C.find_best(w.N, "gradient")
        d_or, bad = O.apply_updates(Io, Jo, check=False)
        C.apply_updates(Io, Jo)
        O.theta_update()
        obj_or = O.objective()
        C.theta_update()
        obj = C.objective()
        assert abs(obj - obj_or) <= 1e-9 * abs(obj_or), (s, obj, obj_or)
        assert obj_or >= prev - 1e-9 * abs(prev)
        prev = obj_or
    C2 = ctx_for(w, lam, "fp32")
    prev = C2.objective()
    for s in range(3):
        st = C2.sweep("gradient")
        assert st["objective"] >= prev - 1e-6 * abs(prev), (s, st, prev)
        prev = st["objective"]
