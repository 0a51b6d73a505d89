"""Python binding of librec.so, the gfx950 library for greedy coordinate
descent network reconstruction (arXiv 2401.01404).

Argument marshalling only: every step of the method runs in the library's
HIP kernels; PyTorch provides device memory and the stream.  There is no CPU
fallback: without the built library (``python -m paper_2401_01404_amd.build``)
or without a GPU every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librec.so")

MODELS = {"ising": 0, "gauss": 1, "kinetic": 2}
PREC = {"fp64": 0, "fp32": 1}
SEARCH = {"nndescent": 0, "exhaustive": 1, "surrogate": 2, "exact_knn": 3, "screen": 4, "gradient": 5}

# every symbol include/rec.h declares
SYMBOLS = ["rec_workspace_size", "rec_create", "rec_destroy", "rec_score_pairs", "rec_find_best_candidates",
           "rec_gcd_sweep", "rec_apply_updates", "rec_theta_update", "rec_objective",
           "rec_get_model", "rec_set_model", "rec_get_fields", "rec_knn", "rec_set_timing",
           "rec_kernel_time", "rec_status_str", "rec_last_error", "rec_sketch", "rec_mlp_params",
           "rec_mlp_infer", "rec_mlp_grad", "rec_mlp_train", "rec_surrogate_config",
           "rec_surrogate_stats", "rec_screen_time", "rec_grad_pairs", "rec_score_pairs_noalloc",
           "rec_cd_sweep", "rec_search_levels"]
SUR_NPARAM = 41345
SUR_SKETCH_DIM = 64
SUR_MAX_BATCH = 8192


class RecConfig(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("xtype", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("knn_k_override", ctypes.c_int32), ("N", ctypes.c_int64), ("M", ctypes.c_int64),
                ("ldx", ctypes.c_int64), ("lam", ctypes.c_double), ("kappa", ctypes.c_double),
                ("nnd_eps", ctypes.c_double), ("nnd_max_iter", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("max_nnz", ctypes.c_int64), ("log2_cache", ctypes.c_int32),
                ("reserved1", ctypes.c_int32)]


class SweepStats(ctypes.Structure):
    _fields_ = [("objective", ctypes.c_double), ("delta", ctypes.c_double),
                ("accepted", ctypes.c_int64), ("n_best", ctypes.c_int64),
                ("pair_evals", ctypes.c_int64), ("nnd_iters", ctypes.c_int64),
                ("levels", ctypes.c_int64), ("rounds", ctypes.c_int64),
                ("t_search_ms", ctypes.c_double), ("t_update_ms", ctypes.c_double),
                ("t_theta_ms", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class RecError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def lib():
    """Load librec.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librec.so is not built: run python -m paper_2401_01404_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        sig = {
            "rec_workspace_size": [ctypes.POINTER(RecConfig), ctypes.POINTER(ctypes.c_size_t)],
            "rec_create": [ctypes.POINTER(RecConfig), vp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)],
            "rec_destroy": [vp],
            "rec_score_pairs": [vp, i64, vp, vp, vp, vp],
            "rec_score_pairs_noalloc": [vp, i64, vp, vp, vp, vp],
            "rec_grad_pairs": [vp, i64, vp, vp, vp],
            "rec_find_best_candidates": [vp, i64, i32, vp, vp, vp, ctypes.POINTER(i64), ctypes.POINTER(SweepStats)],
            "rec_gcd_sweep": [vp, i32, ctypes.POINTER(SweepStats)],
            "rec_cd_sweep": [vp, ctypes.POINTER(SweepStats)],
            "rec_search_levels": [vp, i32, vp, ctypes.POINTER(i32)],
            "rec_apply_updates": [vp, i64, vp, vp, ctypes.POINTER(dbl)],
            "rec_theta_update": [vp, ctypes.POINTER(dbl)],
            "rec_objective": [vp, ctypes.POINTER(dbl)],
            "rec_get_model": [vp, i64, vp, vp, vp, vp, ctypes.POINTER(i64)],
            "rec_set_model": [vp, i64, vp, vp, vp, vp],
            "rec_get_fields": [vp, vp],
            "rec_knn": [vp, i64, vp, i32, i32, i32, vp, vp, ctypes.POINTER(i32)],
            "rec_set_timing": [vp, i32],
            "rec_kernel_time": [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64), ctypes.c_void_p],
            "rec_screen_time": [vp, ctypes.c_void_p],
            "rec_sketch": [vp, vp],
            "rec_mlp_params": [vp, vp, vp],
            "rec_mlp_infer": [vp, i64, vp, vp, vp],
            "rec_mlp_grad": [vp, i64, vp, vp, vp, vp, ctypes.POINTER(dbl)],
            "rec_mlp_train": [vp, i64, vp, vp, vp, i32, ctypes.c_float, ctypes.POINTER(dbl)],
            "rec_surrogate_config": [vp, dbl, dbl, i32, ctypes.c_float, i32, i32],
            "rec_surrogate_stats": [vp, ctypes.POINTER(dbl)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.rec_status_str.argtypes = [ctypes.c_int]
        L.rec_status_str.restype = ctypes.c_char_p
        L.rec_last_error.argtypes = [vp]
        L.rec_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def default_lambda(X, model: str, c: float = 2.0) -> float:
    """lambda = c sqrt(M) median_i v_i with v_i the per-node sample variance
    (1 - mean^2 for +-1 data, mean square for Gaussian data)."""
    X = np.asarray(X)
    if model == "gauss":
        M = X.shape[1]
        v = (X.astype(np.float64) ** 2).mean(axis=1)
    else:
        cols = X[:, 1:] if model == "kinetic" else X
        M = cols.shape[1]
        v = 1.0 - cols.astype(np.float64).mean(axis=1) ** 2
    return float(c * np.sqrt(M) * np.median(v))


class Context:
    """A reconstruction problem living on the GPU.

    X: torch tensor on a GPU, node-major (N rows); int8 +-1 for "ising"
    (N x M) and "kinetic" (N x (T+1)), float32 for "gauss".
    """

    def __init__(self, X, model: str, lam: float, kappa: float = 4.0, prec: str = "fp32",
                 seed: int = 0, nnd_eps: float = 1e-3, nnd_max_iter: int = 0, knn_k: int = 0,
                 max_nnz: int = 0, log2_cache: int = 0):
        import torch
        if not X.is_cuda:
            raise ValueError("X must be a GPU tensor")
        if X.dim() != 2 or X.stride(1) != 1:
            raise ValueError("X must be a 2-D row-major tensor")
        self.torch = torch
        self.device = X.device
        self.model = model
        N = X.shape[0]
        M = X.shape[1] - 1 if model == "kinetic" else X.shape[1]
        cfg = RecConfig()
        cfg.model = MODELS[model]
        cfg.xtype = 1 if X.dtype == torch.float32 else 0
        cfg.prec = PREC[prec]
        cfg.knn_k_override = knn_k
        cfg.N, cfg.M, cfg.ldx = N, M, X.stride(0)
        cfg.lam, cfg.kappa = float(lam), float(kappa)
        cfg.nnd_eps, cfg.nnd_max_iter = nnd_eps, nnd_max_iter
        cfg.seed, cfg.max_nnz, cfg.log2_cache = seed, max_nnz, log2_cache
        self.cfg = cfg
        self.N, self.M = N, M
        L = lib()
        sz = ctypes.c_size_t()
        self._check(L.rec_workspace_size(ctypes.byref(cfg), ctypes.byref(sz)), None)
        self.ws_bytes = sz.value
        self.ws = torch.empty(sz.value, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            self._check(L.rec_create(ctypes.byref(cfg), _ptr(X), _ptr(self.ws), sz.value,
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), None)
        self.h = h
        self.m = max(1, int(np.floor(kappa * N + 0.5)))

    def _check(self, st, h):
        if st != 0:
            L = lib()
            msg = L.rec_last_error(h).decode() if h else ""
            raise RecError(st, f"{L.rec_status_str(st).decode()}: {msg}")

    def close(self):
        if getattr(self, "h", None):
            lib().rec_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _i32(self, a):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device=self.device, dtype=t.int32).contiguous()
        return t.as_tensor(np.asarray(a, np.int32), device=self.device)

    def score_pairs(self, I, J):
        """Exact gains and argmax weights of the pairs (I[p], J[p])."""
        t = self.torch
        I, J = self._i32(I), self._i32(J)
        g = t.empty(len(I), dtype=t.float64, device=self.device)
        w = t.empty(len(I), dtype=t.float64, device=self.device)
        self._check(lib().rec_score_pairs(self.h, len(I), _ptr(I), _ptr(J), _ptr(g), _ptr(w)), self.h)
        return g, w

    def score_pairs_noalloc(self, I, J, gain=None, wopt=None):
        """rec_score_pairs_noalloc: the same scores with the library's static
        scratch (at most 2^20 pairs); writes into gain / wopt when given."""
        t = self.torch
        I, J = self._i32(I), self._i32(J)
        g = gain if gain is not None else t.empty(len(I), dtype=t.float64, device=self.device)
        w = wopt if wopt is not None else t.empty(len(I), dtype=t.float64, device=self.device)
        self._check(lib().rec_score_pairs_noalloc(self.h, len(I), _ptr(I), _ptr(J), _ptr(g), _ptr(w)),
                    self.h)
        return g, w

    def grad_pairs(self, I, J):
        """Gradient distances |dpi/dW_ij| of the pairs (I[p], J[p])."""
        t = self.torch
        I, J = self._i32(I), self._i32(J)
        d = t.empty(len(I), dtype=t.float64, device=self.device)
        self._check(lib().rec_grad_pairs(self.h, len(I), _ptr(I), _ptr(J), _ptr(d)), self.h)
        return d

    def find_best(self, m: int, search: str = "nndescent"):
        t = self.torch
        I = t.empty(m, dtype=t.int32, device=self.device)
        J = t.empty(m, dtype=t.int32, device=self.device)
        G = t.empty(m, dtype=t.float64, device=self.device)
        n = ctypes.c_int64()
        st = SweepStats()
        self._check(lib().rec_find_best_candidates(self.h, m, SEARCH[search], _ptr(I), _ptr(J), _ptr(G),
                                        ctypes.byref(n), ctypes.byref(st)), self.h)
        k = n.value
        return I[:k], J[:k], G[:k], st.as_dict()

    def sweep(self, search: str = "nndescent"):
        st = SweepStats()
        self._check(lib().rec_gcd_sweep(self.h, SEARCH[search], ctypes.byref(st)), self.h)
        return st.as_dict()

    def search_levels(self):
        """Node counts N_t of the levels of the last FindBest search."""
        buf = (ctypes.c_int64 * 64)()
        n = ctypes.c_int32()
        self._check(lib().rec_search_levels(self.h, 64, ctypes.cast(buf, ctypes.c_void_p), ctypes.byref(n)), self.h)
        return [int(buf[l]) for l in range(n.value)]

    def cd_sweep(self):
        """One coordinate-descent sweep [Alg. 1] in round-robin order."""
        st = SweepStats()
        self._check(lib().rec_cd_sweep(self.h, ctypes.byref(st)), self.h)
        return st.as_dict()

    def apply_updates(self, I, J):
        I, J = self._i32(I), self._i32(J)
        d = ctypes.c_double()
        self._check(lib().rec_apply_updates(self.h, len(I), _ptr(I), _ptr(J), ctypes.byref(d)), self.h)
        return d.value

    def theta_update(self):
        o = ctypes.c_double()
        self._check(lib().rec_theta_update(self.h, ctypes.byref(o)), self.h)
        return o.value

    def objective(self):
        o = ctypes.c_double()
        self._check(lib().rec_objective(self.h, ctypes.byref(o)), self.h)
        return o.value

    def get_model(self):
        t = self.torch
        n = ctypes.c_int64()
        th = t.empty(self.N, dtype=t.float64, device=self.device)
        self._check(lib().rec_get_model(self.h, 0, None, None, None, _ptr(th), ctypes.byref(n)), self.h)
        k = n.value
        ei = t.empty(max(k, 1), dtype=t.int32, device=self.device)
        ej = t.empty(max(k, 1), dtype=t.int32, device=self.device)
        w = t.empty(max(k, 1), dtype=t.float64, device=self.device)
        self._check(lib().rec_get_model(self.h, k, _ptr(ei), _ptr(ej), _ptr(w), _ptr(th),
                                        ctypes.byref(n)), self.h)
        return ei[:k], ej[:k], w[:k], th

    def set_model(self, ei, ej, w, theta=None):
        t = self.torch
        ei, ej = self._i32(ei), self._i32(ej)
        w = t.as_tensor(np.asarray(w, np.float64) if not isinstance(w, t.Tensor) else w,
                        dtype=t.float64, device=self.device).contiguous()
        th = None
        if theta is not None:
            th = t.as_tensor(np.asarray(theta, np.float64) if not isinstance(theta, t.Tensor) else theta,
                             dtype=t.float64, device=self.device).contiguous()
        self._check(lib().rec_set_model(self.h, len(ei), _ptr(ei), _ptr(ej), _ptr(w), _ptr(th)), self.h)

    def fields(self):
        t = self.torch
        H = t.empty((self.N, self.M), dtype=t.float64, device=self.device)
        self._check(lib().rec_get_fields(self.h, _ptr(H)), self.h)
        return H

    def knn(self, S, k: int, level: int = 0, mode: str = "nndescent", dist: str = "gain"):
        """KNN lists over S; dist "gradient" (NNDescent only) scores by the
        gradient distance instead of the exact gain."""
        t = self.torch
        S = self._i32(S)
        nbr = t.empty((len(S), k), dtype=t.int32, device=self.device)
        g = t.empty((len(S), k), dtype=t.float64, device=self.device)
        it = ctypes.c_int32()
        if dist == "gradient":
            if mode != "nndescent":
                raise ValueError("the gradient distance runs with NNDescent")
            mode = "gradient"
        self._check(lib().rec_knn(self.h, len(S), _ptr(S), k, level, SEARCH[mode], _ptr(nbr), _ptr(g),
                                  ctypes.byref(it)), self.h)
        return nbr, g, it.value

    # --- learned proposal ---------------------------------------------
    def _f32(self, a):
        t = self.torch
        return t.as_tensor(a, dtype=t.float32).to(self.device).contiguous()

    def sketch(self):
        t = self.torch
        S = t.empty((self.N, SUR_SKETCH_DIM), dtype=t.float32, device=self.device)
        self._check(lib().rec_sketch(self.h, _ptr(S)), self.h)
        return S

    def mlp_params(self, new=None):
        """Current flat parameters (copy); replaces them by `new` when given."""
        t = self.torch
        cur = t.empty(SUR_NPARAM, dtype=t.float32, device=self.device)
        src = None if new is None else self._f32(new)
        self._check(lib().rec_mlp_params(self.h, _ptr(cur), _ptr(src)), self.h)
        return cur

    def mlp_infer(self, I, J):
        t = self.torch
        I, J = self._i32(I), self._i32(J)
        out = t.empty(len(I), dtype=t.float32, device=self.device)
        self._check(lib().rec_mlp_infer(self.h, len(I), _ptr(I), _ptr(J), _ptr(out)), self.h)
        return out

    def mlp_grad(self, I, J, y):
        t = self.torch
        I, J, y = self._i32(I), self._i32(J), self._f32(y)
        g = t.empty(SUR_NPARAM, dtype=t.float32, device=self.device)
        loss = ctypes.c_double()
        self._check(lib().rec_mlp_grad(self.h, len(I), _ptr(I), _ptr(J), _ptr(y), _ptr(g),
                                       ctypes.byref(loss)), self.h)
        return loss.value, g

    def mlp_train(self, I, J, y, steps: int = 1, lr: float = 1e-3):
        I, J, y = self._i32(I), self._i32(J), self._f32(y)
        loss = ctypes.c_double()
        self._check(lib().rec_mlp_train(self.h, len(I), _ptr(I), _ptr(J), _ptr(y), int(steps),
                                        float(lr), ctypes.byref(loss)), self.h)
        return loss.value

    def surrogate_config(self, rho=0.25, recall_min=0.99, train_steps=50, lr=1e-3, audit_log2=4,
                         zero_log2=6):
        self._check(lib().rec_surrogate_config(self.h, float(rho), float(recall_min), int(train_steps),
                                               float(lr), int(audit_log2), int(zero_log2)), self.h)

    def surrogate_stats(self):
        o = (ctypes.c_double * 10)()
        self._check(lib().rec_surrogate_stats(self.h, o), self.h)
        keys = ["mode", "recall", "scored_frac", "pos_kept", "pos_missed", "records_pos",
                "records_zero", "loss", "calls", "rho"]
        return dict(zip(keys, list(o)))

    def set_timing(self, on: bool = True):
        self._check(lib().rec_set_timing(self.h, 1 if on else 0), self.h)

    def screen_time(self):
        """Screening-contraction instrumentation since the last call."""
        o = (ctypes.c_double * 9)()
        self._check(lib().rec_screen_time(self.h, o), self.h)
        keys = ["full_ms", "full_launches", "full_flops", "sample_ms", "sample_launches", "calls",
                "pairs_decided", "rescored", "second_collect"]
        return {k: o[q] for q, k in enumerate(keys)}

    def kernel_time(self):
        """Pair-score kernel time and work since the last call: (ms, launches,
        {"pairs", "moment_passes", "evals", "log_passes", "screened",
        "t_fetches", "i_loads", "bytes"})."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        w = (ctypes.c_int64 * 8)()
        self._check(lib().rec_kernel_time(self.h, ctypes.byref(ms), ctypes.byref(n), w), self.h)
        return ms.value, n.value, {"pairs": w[0], "moment_passes": w[1], "evals": w[2],
                                   "log_passes": w[3], "screened": w[4], "t_fetches": w[5],
                                   "i_loads": w[6], "bytes": w[7]}
