"""rec_score_pairs_noalloc (the entry point whose scratch is the library's
static device array) against rec_score_pairs, through the C ABI: bit-identical
gains and argmax weights on two calls in a row, the second smaller, for every
model, at W = 0 and after a sweep, alternating between two contexts that share
the GPU's array; and the size limit rejected on the host."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _ctx(w, lam, prec):
    import torch
    import paper_2401_01404_amd as rec
    return rec.Context(torch.as_tensor(w.X).cuda(), w.model, lam, prec=prec)


def _pairs(N, n, seed):
    rng = np.random.default_rng(seed)
    I = rng.integers(0, N, n).astype(np.int32)
    J = rng.integers(0, N - 1, n).astype(np.int32)
    J += (J >= I).astype(np.int32)
    order = np.argsort(I, kind="stable")
    return I[order], J[order]


CASES = {
    "ising": lambda: synth.ising_regular(400, 500, 3, 0.4, seed=41),
    "kinetic": lambda: synth.kinetic_er(400, 500, 4.0, 0.3, seed=41),
    "gauss": lambda: synth.gauss_er(400, 200, 4.0, 0.2, 1e-3, seed=41),
}


@pytest.mark.parametrize("model", ["ising", "kinetic", "gauss"])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_equals_score_pairs(model, prec):
    w = CASES[model]()
    lam = oracle.default_lambda(w.X, model)     # dense lambda: many exact solves queued
    A = _ctx(w, lam, prec)
    B = _ctx(w, 1.5 * lam, prec)
    for state in range(2):
        for n, seed in ((60000, 1), (7000, 2)):     # two calls, the second smaller
            I, J = _pairs(w.N, n, seed + 10 * state)
            for C in (A, B):
                g0, w0 = C.score_pairs(I, J)
                g1, w1 = C.score_pairs_noalloc(I, J)
                g0, w0, g1, w1 = (t.cpu().numpy() for t in (g0, w0, g1, w1))
                assert np.array_equal(g0, g1), np.flatnonzero(g0 != g1)[:5]
                assert np.array_equal(w0, w1)
                assert (g0 > 0).sum() > 0
        A.sweep("exhaustive")
        B.sweep("exhaustive")


def test_noalloc_limits():
    import torch
    import paper_2401_01404_amd as rec
    w = CASES["ising"]()
    C = _ctx(w, oracle.default_lambda(w.X, "ising"), "fp32")
    n = (1 << 20) + 1
    I = torch.zeros(n, dtype=torch.int32, device="cuda")
    J = torch.ones(n, dtype=torch.int32, device="cuda")
    with pytest.raises(rec.RecError) as e:
        C.score_pairs_noalloc(I, J)
    assert e.value.status == -1
    # exactly at the limit, and an invalid pair reported as for rec_score_pairs
    g, _ = C.score_pairs_noalloc(I[: 1 << 20], J[: 1 << 20])
    g0, _ = C.score_pairs(I[:4], J[:4])
    assert torch.equal(g[:4], g0)
    with pytest.raises(rec.RecError) as e:
        C.score_pairs_noalloc(np.array([3], np.int32), np.array([3], np.int32))
    assert e.value.status == -1
    g, _ = C.score_pairs_noalloc(np.array([0, 1], np.int32), np.array([1, 2], np.int32))
    g0, _ = C.score_pairs(np.array([0, 1], np.int32), np.array([1, 2], np.int32))
    assert torch.equal(g, g0)
