"""CPU-side checks of the C ABI: the library loads, exports every function
declared in include/rbcg.h, rejects invalid calls before touching a device,
and its host-side quadrature rule agrees with the oracle's (independently
written) rule and with the scalar identity it discretises."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2501_18717_amd", "librbcg.so")


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "rbcg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rbcg_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("librbcg.so is not built; run `python -m paper_2501_18717_amd.build`")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def _header_struct(name):
    src = open(os.path.join(ROOT, "include", "rbcg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    m = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", src)
    assert m, name
    fields = []
    for decl in m.group(1).split(";"):
        decl = decl.strip()
        if not decl:
            continue
        typ, names = decl.split(None, 1)
        for n in names.split(","):
            fields.append((n.strip(), typ))
    return fields


@pytest.mark.parametrize("cname,pyname", [("rbcg_opts", "Opts"), ("rbcg_info", "Info")])
def test_binding_structs_mirror_header(cname, pyname):
    """The ctypes structures of the binding have the header's fields, in order and width."""
    from paper_2501_18717_amd import rbcg
    width = {"int32_t": ctypes.c_int32, "double": ctypes.c_double, "int64_t": ctypes.c_int64,
             "uint64_t": ctypes.c_uint64}
    want = [(n, width[t]) for n, t in _header_struct(cname)]
    got = list(getattr(rbcg, pyname)._fields_)
    assert [n for n, _ in got] == [n for n, _ in want]
    assert [t for _, t in got] == [t for _, t in want]


def test_status_strings_and_version(lib):
    from paper_2501_18717_amd import rbcg
    for code in range(-7, 1):
        assert rbcg.status_string(code)
    assert rbcg.version() >= 10000


def test_null_context_rejected(lib):
    from paper_2501_18717_amd import rbcg
    assert rbcg._destroy(None) == -1
    h = ctypes.c_void_p()
    assert rbcg._op_dense(None, ctypes.byref(h), 8, None, 8, 0) == -1
    info = (rbcg.Info * 1)()
    o = rbcg.opts(3)
    assert rbcg._path(None, None, None, None, 0, 1, None, None, ctypes.byref(o), info) == -1
    assert rbcg._sqrt(None, None, 1, None, None, ctypes.byref(o), info) == -1
    assert rbcg._invsqrt(None, None, 1, None, None, ctypes.byref(o), info) == -1
    assert rbcg._solve(None, 1, None, None, None, None, None, None, None, None) == -1
    assert rbcg._omega_fill(None, 1, 0, 4, 4, None, 4) == -1
    assert rbcg._op_dense_host(None, ctypes.byref(h), 8, None, 8, 4, 0) == -1


@pytest.mark.parametrize("lo,hi,n", [(1e-6, 244.0, 32), (1e-3, 1.0, 16), (3.6e-6, 244.0, 32), (0.5, 2.0, 8)])
def test_library_quadrature_rule(lib, lo, hi, n):
    """The rule the GPU path uses (C++, AGM / Landen Jacobi functions) matches
    the oracle's mpmath rule node by node and integrates sqrt(lambda)."""
    from oracle import quadrature as oq
    from paper_2501_18717_amd import rbcg
    s, w = rbcg.sqrt_rule(lo, hi, n)
    so, wo = oq.sqrt_rule(lo, hi, n)
    assert np.allclose(s, so, rtol=1e-11, atol=0)
    assert np.allclose(w, wo, rtol=1e-11, atol=0)
    lam = np.logspace(np.log10(lo), np.log10(hi), 200)
    approx = sum(wi * lam / (lam + si) for si, wi in zip(s, w))
    assert np.max(np.abs(approx - np.sqrt(lam)) / np.sqrt(lam)) < 1e-11


def test_quadrature_rule_rejects_bad_interval(lib):
    from paper_2501_18717_amd import rbcg
    with pytest.raises(rbcg.RbcgError):
        rbcg.sqrt_rule(0.0, 1.0, 8)
    with pytest.raises(rbcg.RbcgError):
        rbcg.sqrt_rule(2.0, 1.0, 8)
