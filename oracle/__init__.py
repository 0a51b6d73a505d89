"""ctypes front end of the FP64 CPU oracle (``oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; the GPU library never uses it.
Everything here is argument marshalling; the arithmetic is in ``oracle.cpp``.

Pins that tie the oracle to the paper rather than to itself live in
``tests/test_oracle_pins.py``.  Functions without such a pin are marked
"parity unpinned" in their docstring.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

MODELS = {"ising": 0, "gauss": 1, "kinetic": 2}


# -ffp-contract=off: no fused multiply-adds, so every build rounds the same
# way whatever the target's instruction set.
_FLAGS = ["-O3", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c++17"]


def build(force: bool = False) -> str:
    """Compile oracle.cpp with g++ (-O3, OpenMP, x86-64-v3: AVX2 hosts) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++"] + _FLAGS + ["-march=x86-64-v3", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def use_native() -> str:
    """Rebuild the oracle for this host's CPU (-march=native, same arithmetic:
    no contraction) and load that build; call before the first Oracle is made.
    Used by the CPU-baseline timing, which runs on the host that measures it."""
    global _LIB, _lib
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    path = os.path.join(_HERE, "liboracle_native.so")
    tmp = path + ".tmp%d" % os.getpid()
    subprocess.check_call(["g++"] + _FLAGS + ["-march=native", "-o", tmp, _SRC])
    os.replace(tmp, path)
    _LIB = path
    return path


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use (OMP_NUM_THREADS, else
    the CPUs this process may run on)."""
    v = os.environ.get("OMP_NUM_THREADS", "")
    if v.strip().isdigit() and int(v) > 0:
        return int(v)
    return len(os.sched_getaffinity(0))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _L():
    global _lib
    if _lib is None:
        if _LIB.endswith("liboracle.so"):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, i32, u64, dbl, vp, ci = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                      ctypes.c_double, ctypes.c_void_p, ctypes.c_int)
        sig = {
            "orc_create": (vp, [ci, i64, i64, ci, vp, i64, dbl]),
            "orc_destroy": (None, [vp]),
            "orc_set_model": (None, [vp, i64, vp, vp, vp, vp]),
            "orc_get_model": (i64, [vp, i64, vp, vp, vp, vp]),
            "orc_objective": (dbl, [vp]),
            "orc_node_loglik": (dbl, [vp, i64]),
            "orc_fields": (None, [vp, vp]),
            "orc_theta_update": (None, [vp]),
            "orc_score_pairs": (None, [vp, i64, vp, vp, vp, vp]),
            "orc_pair_deriv": (dbl, [vp, i32, i32, dbl]),
            "orc_find_best": (i64, [vp, i64, ci, u64, dbl, ci, vp, vp, vp, vp]),
            "orc_knn": (ci, [vp, i64, vp, ci, ci, u64, ci, dbl, ci, vp, vp]),
            "orc_knn_init": (None, [i64, i64, ci, u64, ci, ci, vp]),
            "orc_apply_updates": (dbl, [vp, i64, vp, vp, ci, vp]),
            "orc_gcd_sweep": (dbl, [vp, i64, ci, u64, dbl, ci, vp, vp]),
            "orc_cd_sweep": (dbl, [vp]),
            "orc_cd_sweep_order": (dbl, [vp, ci]),
            "orc_lcosh": (dbl, [dbl]),
            "orc_dlcosh": (dbl, [dbl, dbl]),
            "orc_ctr": (u64, [u64, u64, u64, u64]),
            "orc_set_dist": (None, [vp, ci]),
            "orc_grad_pairs": (None, [vp, i64, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, np.int32)


class Oracle:
    """One reconstruction problem held by the CPU oracle.

    model: "ising" (symmetric W, X int8 +-1 N x M), "gauss" (symmetric W,
    X float32 N x M) or "kinetic" (directed W, X int8 N x (T+1), M = T).
    """

    def __init__(self, X: np.ndarray, model: str, lam: float):
        self.model = model
        X = np.ascontiguousarray(X)
        self.N = X.shape[0]
        self.M = X.shape[1] - 1 if model == "kinetic" else X.shape[1]
        xtype = 1 if X.dtype == np.float32 else 0
        if xtype == 0 and X.dtype != np.int8:
            raise TypeError("X must be int8 (+-1) or float32")
        self._X = X
        self.lam = float(lam)
        self.h = _L().orc_create(MODELS[model], self.N, self.M, xtype, _p(X), X.shape[1], self.lam)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            try:
                _lib.orc_destroy(h)
            except Exception:
                pass
            self.h = None

    # --- state ---------------------------------------------------------
    def set_model(self, ei, ej, w, theta=None):
        ei, ej = _i32(ei), _i32(ej)
        w = np.ascontiguousarray(w, np.float64)
        th = None if theta is None else np.ascontiguousarray(theta, np.float64)
        _L().orc_set_model(self.h, len(ei), _p(ei), _p(ej), _p(w), _p(th))

    def get_model(self):
        n = _L().orc_get_model(self.h, 0, None, None, None, None)
        ei = np.zeros(n, np.int32)
        ej = np.zeros(n, np.int32)
        w = np.zeros(n, np.float64)
        th = np.zeros(self.N, np.float64)
        _L().orc_get_model(self.h, n, _p(ei), _p(ej), _p(w), _p(th))
        return ei, ej, w, th

    def objective(self) -> float:
        return _L().orc_objective(self.h)

    def node_loglik(self, i: int) -> float:
        return _L().orc_node_loglik(self.h, i)

    def fields(self) -> np.ndarray:
        H = np.zeros((self.N, self.M), np.float64)
        _L().orc_fields(self.h, _p(H))
        return H

    def theta_update(self):
        _L().orc_theta_update(self.h)

    # --- scores --------------------------------------------------------
    def score_pairs(self, I, J):
        I, J = _i32(I), _i32(J)
        g = np.zeros(len(I), np.float64)
        w = np.zeros(len(I), np.float64)
        _L().orc_score_pairs(self.h, len(I), _p(I), _p(J), _p(g), _p(w))
        return g, w

    def pair_deriv(self, i, j, w):
        return _L().orc_pair_deriv(self.h, int(i), int(j), float(w))

    def grad_pairs(self, I, J):
        """Absolute gradient of the objective in W_ij at the current state
        (the gradient distance of the paper's appendix; central difference at
        the L1 kink), per pair."""
        I, J = _i32(I), _i32(J)
        g = np.zeros(len(I), np.float64)
        _L().orc_grad_pairs(self.h, len(I), _p(I), _p(J), _p(g))
        return g

    def _dist(self, dist):
        _L().orc_set_dist(self.h, {"gain": 0, "gradient": 1}[dist])

    # --- search --------------------------------------------------------
    def find_best(self, m, mode="exhaustive", seed=0, eps=1e-3, max_iter=0, dist="gain"):
        """Best m pairs under the search distance ("gain": the exact gain;
        "gradient": the absolute gradient, see grad_pairs)."""
        mode_id = {"exhaustive": 0, "exact_knn": 1, "nndescent": 2}[mode]
        I = np.zeros(m, np.int32)
        J = np.zeros(m, np.int32)
        G = np.zeros(m, np.float64)
        st = np.zeros(64, np.int64)
        self._dist(dist)
        try:
            n = _L().orc_find_best(self.h, m, mode_id, seed, eps, max_iter, _p(I), _p(J), _p(G), _p(st))
        finally:
            self._dist("gain")
        levels = int(st[0])
        stats = dict(levels=levels, nnd_iters=int(st[1]), evals=int(st[2]),
                     level_n=[int(st[3 + 2 * l]) for l in range(min(levels, 30))],
                     level_k=[int(st[4 + 2 * l]) for l in range(min(levels, 30))])
        return I[:n], J[:n], G[:n], stats

    def knn(self, S, k, mode="nndescent", seed=0, level=0, eps=1e-3, max_iter=0, dist="gain"):
        S = _i32(S)
        J = np.zeros(len(S) * k, np.int32)
        G = np.zeros(len(S) * k, np.float64)
        self._dist(dist)
        try:
            it = _L().orc_knn(self.h, len(S), _p(S), k, {"exact": 1, "nndescent": 2}[mode], seed, level,
                              eps, max_iter, _p(J), _p(G))
        finally:
            self._dist("gain")
        return J.reshape(len(S), k), G.reshape(len(S), k), it

    # --- updates -------------------------------------------------------
    def apply_updates(self, I, J, check=False):
        I, J = _i32(I), _i32(J)
        bad = np.zeros(1, np.int64)
        d = _L().orc_apply_updates(self.h, len(I), _p(I), _p(J), int(check), _p(bad))
        return d, int(bad[0])

    def gcd_sweep(self, m, mode="exhaustive", seed=0, eps=1e-3, max_iter=0, dist="gain"):
        """One GCD sweep; E_best ranked by the search distance, every update
        the exact coordinate maximum."""
        mode_id = {"exhaustive": 0, "exact_knn": 1, "nndescent": 2}[mode]
        obj = np.zeros(1)
        nb = np.zeros(1, np.int64)
        self._dist(dist)
        try:
            d = _L().orc_gcd_sweep(self.h, m, mode_id, seed, eps, max_iter, _p(obj), _p(nb))
        finally:
            self._dist("gain")
        return d, float(obj[0])

    def cd_sweep(self, order="rows"):
        """One CD sweep [Alg. 1] (every coordinate once, then theta); order
        "rows" (index order) or "round_robin" (the node-disjoint rounds of the
        circle method).  Returns sum |dW|."""
        return _L().orc_cd_sweep_order(self.h, {"rows": 0, "round_robin": 1}[order])


def knn_init(n, a, k, seed, level, gid):
    out = np.zeros(k, np.int32)
    _L().orc_knn_init(n, a, k, seed, level, gid, _p(out))
    return out


def lcosh(x):
    return _L().orc_lcosh(float(x))


def dlcosh(a, d):
    return _L().orc_dlcosh(float(a), float(d))


def ctr(seed, stream, a, b):
    return int(_L().orc_ctr(seed, stream, a, b))


def default_lambda(X: np.ndarray, model: str, c: float = 2.0) -> float:
    """Penalty lambda = c * sqrt(M) * median_i v_i (v_i: per-node sample variance:
    1 - mean(x_i)^2 for +-1 data, ||x_i||^2 / M for Gaussian data).  The paper
    leaves lambda to the user ("chosen to achieve a desired level of sparsity")."""
    if model == "gauss":
        M = X.shape[1]
        v = (X.astype(np.float64) ** 2).mean(axis=1)
    else:
        cols = X[:, 1:] if model == "kinetic" else X
        M = cols.shape[1]
        v = 1.0 - cols.astype(np.float64).mean(axis=1) ** 2
    return float(c * np.sqrt(M) * np.median(v))
