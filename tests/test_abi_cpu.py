"""The C-ABI library loads, exports every symbol its headers declare, and
rejects invalid input before touching a device (no GPU needed)."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2406_13191_amd", "libdcopf_dual.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def _declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"\b(dcopf_\w+)\s*\(", txt):
            names.add(m.group(1))
    return sorted(names)


def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = _declared_symbols()
    assert "dcopf_dual_create" in names and "dcopf_dual_solve" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def _tiny():
    from paper_2406_13191_amd import synth
    return synth.make_problem("tiny30", 1)


@pytest.mark.parametrize("mutate,msg", [
    (lambda p: p.replace(f_max=-p.f_max), "f_max"),
    (lambda p: p.replace(p_min=p.p_max + 1), "p_min > p_max"),
    (lambda p: p.replace(q=-np.ones(p.n_gen)), "q < 0"),
    (lambda p: p.replace(gen_bus=np.full(p.n_gen, 99, np.int32)), "gen_bus"),
    (lambda p: p.replace(slack=-1), "slack"),
    (lambda p: p.replace(c=np.full(p.n_gen, np.nan)), "non-finite"),
    (lambda p: p.replace(H=np.where(np.arange(p.n_bus)[None, :] == 0, 1.0, p.H)), "slack"),
])
def test_invalid_inputs(mutate, msg):
    from paper_2406_13191_amd import _abi
    with pytest.raises(_abi.DcopfError) as e:
        _abi.DualSolver(mutate(_tiny()))
    assert e.value.status == -1
    assert msg in str(e.value)


def test_infeasible_load():
    from paper_2406_13191_amd import _abi
    p = _tiny()
    with pytest.raises(_abi.DcopfError) as e:
        _abi.DualSolver(p.replace(d=p.d * 10))
    assert e.value.status == -5


@pytest.mark.parametrize("kw", [dict(alpha=0.0), dict(rho=1.0), dict(rule="adam", beta1=1.0),
                                dict(rule="adagrad", eps=0.0), dict(decay=-1.0),
                                dict(graph_iters=-1)])
def test_invalid_options(kw):
    from paper_2406_13191_amd import _abi
    with pytest.raises(_abi.DcopfError) as e:
        _abi.DualSolver(_tiny(), **kw)
    assert e.value.status == -1


def test_destroy_null_is_noop():
    from paper_2406_13191_amd import _abi
    _abi.lib.dcopf_dual_destroy(None)
    assert _abi.lib.dcopf_dual_step(None, 1) == -1


def test_set_allocator_needs_both_functions_or_neither():
    lib = ctypes.CDLL(LIB)
    alloc_t = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
    free_t = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                              ctypes.c_void_p)
    lib.dcopf_set_allocator.restype = ctypes.c_int
    lib.dcopf_set_allocator.argtypes = [alloc_t, free_t, ctypes.c_void_p]
    a = alloc_t(lambda n, s, c: None)
    f = free_t(lambda p, n, s, c: None)
    assert lib.dcopf_set_allocator(a, free_t(), None) == -1
    assert lib.dcopf_set_allocator(alloc_t(), f, None) == -1
    assert lib.dcopf_set_allocator(a, f, None) == 0
    assert lib.dcopf_set_allocator(alloc_t(), free_t(), None) == 0
