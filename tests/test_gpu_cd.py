"""The coordinate-descent baseline [Alg. 1] on the GPU against the FP64
oracle's CD in the same round-robin visiting order: every coupling, theta and
the objective after each sweep, for the three models, an odd N (a phantom node
in the schedule) and an even N, FP64 and FP32."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _case(model, N):
    if model == "gauss":
        return synth.gauss_er(N, 80, 3.0, 0.2, 1e-3, seed=51)
    if model == "kinetic":
        return synth.kinetic_er(N, 300, 3.0, 0.5, seed=51)
    return synth.ising_er(N, 200, 3.0, 0.5, 0.1, seed=51)


def _dense(ei, ej, w, N, directed):
    W = np.zeros((N, N))
    W[ei, ej] = w
    if not directed:
        W = W + W.T
    return W


@pytest.mark.parametrize("model", ["ising", "gauss", "kinetic"])
@pytest.mark.parametrize("N", [37, 64])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cd_sweeps_match_oracle(model, N, prec):
    import torch
    import paper_2401_01404_amd as rec
    w = _case(model, N)
    lam = oracle.default_lambda(w.X, model, c=1.0)
    C = rec.Context(torch.as_tensor(w.X).cuda(), model, lam, prec=prec)
    O = oracle.Oracle(w.X, model, lam)
    tol = 1e-9 if prec == "fp64" else 2e-5
    for sweep in range(3):
        st = C.cd_sweep()
        d = O.cd_sweep("round_robin")
        obj = O.objective()
        assert abs(st["objective"] - obj) <= tol * abs(obj), (sweep, st["objective"], obj)
        assert abs(st["delta"] - d) <= tol * 10 * max(1.0, d), (sweep, st["delta"], d)
        assert st["rounds"] == N + (N & 1) - 1
        ei, ej, wv, th = (t.cpu().numpy() for t in C.get_model())
        oi, oj, ov, oth = O.get_model()
        Wg = _dense(ei, ej, wv, N, model == "kinetic")
        Wo = _dense(oi, oj, ov, N, model == "kinetic")
        scale = max(1.0, np.abs(Wo).max())
        assert np.abs(Wg - Wo).max() <= (1e-9 if prec == "fp64" else 1e-4) * scale
        assert np.abs(th - oth).max() <= (1e-9 if prec == "fp64" else 1e-4) * max(1.0, np.abs(oth).max())
        assert len(ei) > 0


def test_cd_then_gcd_reach_the_same_optimum():
    """CD and GCD converge to the same optimum of the convex objective."""
    import torch
    import paper_2401_01404_amd as rec
    w = _case("ising", 40)
    lam = oracle.default_lambda(w.X, "ising", c=1.0)
    A = rec.Context(torch.as_tensor(w.X).cuda(), "ising", lam, prec="fp64", kappa=1.0)
    B = rec.Context(torch.as_tensor(w.X).cuda(), "ising", lam, prec="fp64", kappa=1.0)
    for _ in range(200):
        if A.cd_sweep()["delta"] < 1e-12:
            break
    for _ in range(400):
        if B.sweep("exhaustive")["delta"] < 1e-12:
            break
    oa, ob = A.objective(), B.objective()
    assert abs(oa - ob) <= 1e-10 * abs(oa), (oa, ob)
