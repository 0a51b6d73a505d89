"""Seeded synthetic workloads shared by the GPU tests, the oracle tests and the bench.

Only generative models live here (random graphs, weights, Gibbs / Glauber /
Gaussian samplers); none of the reconstruction method's arithmetic does.
Every array is produced by ``synth.c`` from counter-based SplitMix64 draws,
so a workload is a pure function of its parameters and seed.

Data layout: node-major ``X[i, m]`` (row i holds the samples of node i).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None

# Random streams of the weight / field draws (the graph and sampler streams
# are fixed inside synth.c).
ST_WEIGHT = 2
ST_THETA = 9


def build(force: bool = False) -> str:
    """Compile synth.c into libsynth.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, i32, u64, dbl, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
        lib.synth_er_undirected.restype = i64
        lib.synth_er_undirected.argtypes = [i64, dbl, u64, i64, vp, vp]
        lib.synth_er_directed.restype = i64
        lib.synth_er_directed.argtypes = [i64, dbl, u64, i64, vp, vp]
        lib.synth_regular.restype = i64
        lib.synth_regular.argtypes = [i64, ctypes.c_int, u64, ctypes.c_int, vp, vp]
        lib.synth_normal.restype = None
        lib.synth_normal.argtypes = [i64, dbl, dbl, u64, u64, vp]
        lib.synth_uniform.restype = None
        lib.synth_uniform.argtypes = [i64, dbl, dbl, u64, u64, vp]
        lib.synth_gibbs.restype = ctypes.c_int
        lib.synth_gibbs.argtypes = [i64, i64, i64, vp, vp, vp, vp, i64, i64, u64, vp, i64]
        lib.synth_glauber.restype = ctypes.c_int
        lib.synth_glauber.argtypes = [i64, i64, i64, vp, vp, vp, vp, u64, vp, i64]
        lib.synth_gauss.restype = ctypes.c_int
        lib.synth_gauss.argtypes = [i64, i64, i64, vp, vp, vp, dbl, u64, dbl, i64, vp, i64, vp]
        lib.synth_ctr.restype = u64
        lib.synth_ctr.argtypes = [u64, u64, u64, u64]
        lib.synth_mix64.restype = u64
        lib.synth_mix64.argtypes = [u64]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ------------------------------------------------------------------ graphs --

def er_undirected(N: int, mean_deg: float, seed: int):
    """G(N, p) with p = mean_deg / (N - 1); returns (ei, ej) int32 with ei < ej."""
    p = mean_deg / (N - 1)
    cap = int(N * mean_deg / 2 * 1.2 + 64)
    while True:
        ei = np.zeros(cap, np.int32)
        ej = np.zeros(cap, np.int32)
        n = _L().synth_er_undirected(N, p, seed, cap, _p(ei), _p(ej))
        if n <= cap:
            return ei[:n].copy(), ej[:n].copy()
        cap = n


def er_directed(N: int, mean_out: float, seed: int):
    """Directed G(N, p), p = mean_out / (N - 1) per ordered pair; returns (dst, src)."""
    p = mean_out / (N - 1)
    cap = int(N * mean_out * 1.2 + 64)
    while True:
        d = np.zeros(cap, np.int32)
        s = np.zeros(cap, np.int32)
        n = _L().synth_er_directed(N, p, seed, cap, _p(d), _p(s))
        if n <= cap:
            return d[:n].copy(), s[:n].copy()
        cap = n


def regular(N: int, d: int, seed: int, max_tries: int = 1000):
    """Random simple d-regular graph (configuration model with redraws)."""
    E = N * d // 2
    ei = np.zeros(E, np.int32)
    ej = np.zeros(E, np.int32)
    n = _L().synth_regular(N, d, seed, max_tries, _p(ei), _p(ej))
    if n < 0:
        raise RuntimeError("no simple %d-regular pairing found" % d)
    return ei, ej


def normal(n: int, mu: float, sigma: float, seed: int, stream: int) -> np.ndarray:
    out = np.zeros(n, np.float64)
    _L().synth_normal(n, mu, sigma, seed, stream, _p(out))
    return out


def uniform(n: int, lo: float, hi: float, seed: int, stream: int) -> np.ndarray:
    out = np.zeros(n, np.float64)
    _L().synth_uniform(n, lo, hi, seed, stream, _p(out))
    return out


# ---------------------------------------------------------------- samplers --

def gibbs(N, M, ei, ej, w, theta, burn=1000, thin=10, seed=0) -> np.ndarray:
    """Equilibrium Ising samples, node-major int8 (N, M) of +-1."""
    X = np.zeros((N, M), np.int8)
    ei = np.ascontiguousarray(ei, np.int32)
    ej = np.ascontiguousarray(ej, np.int32)
    w = np.ascontiguousarray(w, np.float64)
    th = None if theta is None else np.ascontiguousarray(theta, np.float64)
    rc = _L().synth_gibbs(N, M, len(ei), _p(ei), _p(ej), _p(w), None if th is None else _p(th),
                          burn, thin, seed, _p(X), M)
    if rc != 0:
        raise RuntimeError("synth_gibbs failed")
    return X


def glauber(N, T, dst, src, w, theta, seed=0) -> np.ndarray:
    """Kinetic Ising series, node-major int8 (N, T+1) of +-1 (columns t = 0..T)."""
    X = np.zeros((N, T + 1), np.int8)
    dst = np.ascontiguousarray(dst, np.int32)
    src = np.ascontiguousarray(src, np.int32)
    w = np.ascontiguousarray(w, np.float64)
    th = None if theta is None else np.ascontiguousarray(theta, np.float64)
    rc = _L().synth_glauber(N, T, len(dst), _p(dst), _p(src), _p(w), None if th is None else _p(th),
                            seed, _p(X), T + 1)
    if rc != 0:
        raise RuntimeError("synth_glauber failed")
    return X


def gauss(N, M, ei, ej, off, eps=1e-3, seed=0, tol=1e-12, max_iter=100000):
    """x ~ N(0, Theta^{-1}); returns (X float32 (N, M), Theta diagonal)."""
    X = np.zeros((N, M), np.float32)
    diag = np.zeros(N, np.float64)
    ei = np.ascontiguousarray(ei, np.int32)
    ej = np.ascontiguousarray(ej, np.int32)
    off = np.ascontiguousarray(off, np.float64)
    rc = _L().synth_gauss(N, M, len(ei), _p(ei), _p(ej), _p(off), eps, seed, tol, max_iter,
                          _p(X), M, _p(diag))
    if rc < 0:
        raise RuntimeError("synth_gauss: CG did not converge")
    return X, diag


def ctr(seed: int, stream: int, a: int, b: int) -> int:
    return int(_L().synth_ctr(seed, stream, a, b))


# ------------------------------------------------------------------ lambda --

def sparsity_lambda(X, model: str, q: float | None = None) -> float:
    """The L1 penalty of a workload, set for a target sparsity (the appendix
    on the Ising model leaves lambda to the user, to be picked for the
    sparsity it gives).

    At W = 0 the derivative of the objective change in one coupling between
    two independent nodes is a sum of M independent zero-mean terms: Ising
    f'(0) = 2 sum_m (x_im - xbar_i)(x_jm - xbar_j), standard deviation
    2 sqrt(M v_i v_j); Gaussian a = -2 x_i . x_j, 2 sqrt(M v_i v_j) with
    v = ||x||^2 / M; kinetic f'(0) = sum_t (x_{i,t} - xbar_i) x_{j,t-1},
    sqrt(T v_i).  With sigma that deviation at the median v, lambda =
    sigma sqrt(2 ln(P / q)) for P coordinates (N(N-1)/2 symmetric, N(N-1)
    directed) puts the expected number of such pairs whose gain is positive
    at W = 0 (|f'(0)| > lambda, a two-sided normal tail) at most q; the
    default q = N.  Pairs of truly coupled nodes (and their indirect
    correlations) pass in addition, so the couplings found stay O(N)
    instead of growing by about m each sweep."""
    X = np.asarray(X)
    N = X.shape[0]
    if model == "gauss":
        M = X.shape[1]
        v = np.median((X.astype(np.float64) ** 2).mean(axis=1))
        sigma = 2.0 * np.sqrt(M) * v
        P = N * (N - 1) / 2.0
    elif model == "ising":
        M = X.shape[1]
        v = np.median(1.0 - X.astype(np.float64).mean(axis=1) ** 2)
        sigma = 2.0 * np.sqrt(M) * v
        P = N * (N - 1) / 2.0
    elif model == "kinetic":
        M = X.shape[1] - 1
        v = np.median(1.0 - X[:, 1:].astype(np.float64).mean(axis=1) ** 2)
        sigma = np.sqrt(M * v)
        P = float(N) * (N - 1)
    else:
        raise KeyError(model)
    q = float(N) if q is None else float(q)
    return float(sigma * np.sqrt(2.0 * np.log(max(P / q, np.e))))


# --------------------------------------------------------------- workloads --

@dataclass
class Workload:
    """A generated problem: data X plus the ground truth that produced it."""
    name: str
    model: str              # "ising", "kinetic" or "gauss"
    X: np.ndarray           # node-major data, int8 +-1 or float32
    ei: np.ndarray          # ground-truth edges (ising/gauss: ei<ej; kinetic: dst)
    ej: np.ndarray          # (kinetic: src)
    w: np.ndarray           # ground-truth couplings / off-diagonal precisions
    theta: np.ndarray | None = None
    params: dict = field(default_factory=dict)

    @property
    def N(self):
        return self.X.shape[0]

    @property
    def M(self):
        """Number of likelihood terms per node: samples, or transitions for kinetic."""
        return self.X.shape[1] - 1 if self.model == "kinetic" else self.X.shape[1]


def ising_er(N, M, mean_deg=3.0, w_sigma=0.25, theta_sigma=0.1, burn=1000, thin=10, seed=0,
             name="ising_er"):
    ei, ej = er_undirected(N, mean_deg, seed)
    w = normal(len(ei), 0.0, w_sigma, seed, ST_WEIGHT)
    theta = normal(N, 0.0, theta_sigma, seed, ST_THETA) if theta_sigma > 0 else np.zeros(N)
    X = gibbs(N, M, ei, ej, w, theta, burn, thin, seed)
    return Workload(name, "ising", X, ei, ej, w, theta,
                    dict(N=N, M=M, graph="er", mean_deg=mean_deg, w_sigma=w_sigma,
                         theta_sigma=theta_sigma, burn=burn, thin=thin, seed=seed))


def ising_regular(N, M, d=3, w_max=0.4, burn=1000, thin=10, seed=0, name="ising_regular"):
    ei, ej = regular(N, d, seed)
    w = uniform(len(ei), -w_max, w_max, seed, ST_WEIGHT)
    theta = np.zeros(N)
    X = gibbs(N, M, ei, ej, w, theta, burn, thin, seed)
    return Workload(name, "ising", X, ei, ej, w, theta,
                    dict(N=N, M=M, graph="regular", d=d, w_max=w_max, burn=burn, thin=thin, seed=seed))


def kinetic_er(N, T, mean_out=5.0, w_sigma=0.3, seed=0, name="kinetic_er"):
    dst, src = er_directed(N, mean_out, seed)
    w = normal(len(dst), 0.0, w_sigma, seed, ST_WEIGHT)
    theta = np.zeros(N)
    X = glauber(N, T, dst, src, w, theta, seed)
    return Workload(name, "kinetic", X, dst, src, w, theta,
                    dict(N=N, T=T, graph="directed_er", mean_out=mean_out, w_sigma=w_sigma, seed=seed))


def gauss_scaling(N, M=10, mean_deg=5.0, mean=-1e3, sd=10.0, eps=1e-3, seed=0, name="gauss_scaling"):
    """The FindBest runtime study's problems [Sec. 5, the runtime figure]: an ER
    graph of mean degree 5, off-diagonal precisions ~ N(-1000, 10^2), diagonal
    sum_j |W_ij| / (1 - eps)^2 with eps = 1e-3, M = 10 samples."""
    ei, ej = er_undirected(N, mean_deg, seed)
    off = normal(len(ei), mean, sd, seed, ST_WEIGHT)
    X, diag = gauss(N, M, ei, ej, off, eps, seed)
    return Workload(name, "gauss", X, ei, ej, off, diag,
                    dict(N=N, M=M, graph="er", mean_deg=mean_deg, off_mean=mean, off_sd=sd, eps=eps,
                         seed=seed))


def gauss_er(N, M, mean_deg=4.0, off_max=0.2, eps=1e-3, seed=0, name="gauss_er"):
    ei, ej = er_undirected(N, mean_deg, seed)
    off = uniform(len(ei), -off_max, off_max, seed, ST_WEIGHT)
    X, diag = gauss(N, M, ei, ej, off, eps, seed)
    return Workload(name, "gauss", X, ei, ej, off, diag,
                    dict(N=N, M=M, graph="er", mean_deg=mean_deg, off_max=off_max, eps=eps, seed=seed))


def config(cid: str, scale: float = 1.0) -> Workload:
    """The five benchmark workloads at full size (scale=1) or with N scaled down.

    C1  Ising, ER mean degree 3, w~N(0,0.25^2), theta~N(0,0.1^2), N=100, M=500
    C2  Ising, random 3-regular, w~U[-0.4,0.4], N=10^4, M=1000
    C3  Gaussian, ER mean degree 4, offdiag U[-0.2,0.2], N=2*10^4, M=200
    C4  kinetic Ising, directed ER mean out-degree 5, w~N(0,0.3^2), N=10^5, T=1000
    C4s Ising, C2's generator (random 3-regular, w~U[-0.4,0.4]) at N=10^5, M=1000
    C5  Ising, ER mean degree 3, w~N(0,0.3^2), N=10^6, M=100
    Gibbs chains: 1000 burn-in sweeps, 10 sweeps between samples, seed 0.
    """
    def n(v):
        return max(8, int(round(v * scale)))
    if cid == "C1":
        return ising_er(n(100), 500, 3.0, 0.25, 0.1, name="C1")
    if cid == "C2":
        N = n(10_000)
        N += N % 2
        return ising_regular(N, 1000, 3, 0.4, name="C2")
    if cid == "C3":
        return gauss_er(n(20_000), 200, 4.0, 0.2, 1e-3, name="C3")
    if cid == "C4":
        return kinetic_er(n(100_000), 1000, 5.0, 0.3, name="C4")
    if cid == "C4s":
        N = n(100_000)
        N += N % 2
        return ising_regular(N, 1000, 3, 0.4, name="C4s")
    if cid == "C5":
        return ising_er(n(1_000_000), 100, 3.0, 0.3, 0.0, name="C5")
    raise KeyError(cid)
