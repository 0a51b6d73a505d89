"""The C ABI on the CPU: the library loads, exports every function the header
declares, and the host-only workspace planner validates configurations."""
import ctypes
import os
import re

import pytest

import paper_2401_01404_amd as rec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rec.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rec_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_symbols():
    assert set(declared_functions()) == set(rec.SYMBOLS)


def test_library_exports_every_declared_symbol():
    L = rec.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def cfg(**kw):
    c = rec.RecConfig()
    c.model, c.xtype, c.prec = 0, 0, 1
    c.N, c.M, c.ldx = 1000, 300, 300
    c.lam, c.kappa, c.nnd_eps = 10.0, 4.0, 1e-3
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def wsize(c):
    sz = ctypes.c_size_t()
    st = rec.lib().rec_workspace_size(ctypes.byref(c), ctypes.byref(sz))
    return st, sz.value


def test_workspace_size_valid_configs():
    for kw in [{}, dict(prec=0), dict(model=2, ldx=301), dict(model=1, xtype=1), dict(M=2048, ldx=2048),
               dict(N=2, M=1, ldx=1)]:
        st, sz = wsize(cfg(**kw))
        assert st == 0, kw
        assert sz > 0
    # FP64 needs more room than FP32
    assert wsize(cfg(prec=0))[1] > wsize(cfg(prec=1))[1]


@pytest.mark.parametrize("kw", [dict(N=1), dict(N=(1 << 20) + 1), dict(M=0), dict(M=2049, ldx=2049),
                                dict(model=3), dict(model=1), dict(xtype=1), dict(prec=2),
                                dict(ldx=299), dict(model=2, ldx=300), dict(lam=-1.0),
                                dict(lam=float("nan")), dict(kappa=0.0), dict(log2_cache=31)])
def test_workspace_size_rejects_bad_configs(kw):
    st, _ = wsize(cfg(**kw))
    assert st == -1, kw


def test_null_arguments_rejected():
    L = rec.lib()
    c = cfg()
    assert L.rec_workspace_size(None, None) == -1
    assert L.rec_workspace_size(ctypes.byref(c), None) == -1
    h = ctypes.c_void_p()
    assert L.rec_create(ctypes.byref(c), None, None, 0, None, ctypes.byref(h)) == -1
    assert L.rec_destroy(None) == -1
    assert L.rec_status_str(-2) == b"workspace too small"
